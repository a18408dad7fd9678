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

// Extreme coordinates of the body turned by theta0 about the pose origin, and the first
// vertices attaining them.  A body that does not turn is only translated: rounding is
// monotone, so each posed extreme is the turned extreme plus the translation, rounded, and
// is attained at the same vertex (a vertex that ties with it after rounding is an extreme
// as well).  mag: the largest of their magnitudes.
struct Extremes {
    double xlo, xhi, ylo, yhi, mag;
    int il, ir, ib, it;
};

// True when a translation from c0 to c1 surely moves every vertex by less than h along
// that axis, the rounding of the posed coordinates included (mag: the turned body's
// largest coordinate magnitude); false means: check the vertices one by one.
__host__ __device__ inline bool surely_within(double c0, double c1, double h, double mag) {
    double d = fabs(c1 - c0);
    double C = fmax(fabs(c0), fabs(c1));
    return d + 0x1p-49 * (mag + C + d) < h;
}

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
    Extremes ext0;    // its extreme coordinates
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
    int remaining;    // steps still to plan in this run
    Box lbox[3];
    Level lev[3];
    Motion mot;
    Box last_sweep_box;
    // a turning body's angle terms at time trig_t (the end of the last planned step, the
    // start of the next): sin and cos of omega t, and cos and sin of the pose angle there;
    // trig_ok = 0 (as the host writes it) means none
    int trig_ok;
    double trig_t, sin_w, cos_w, cs_th, sn_th;
};

__device__ inline Pose pose_at_dev(const PlanConst& P, double t) {
    if (P.amp == 0.0) return Pose{P.cs0, P.sn0, P.ref_x + P.vx * t, P.ref_y + P.vy * t};
    double th = P.theta0 + P.amp * sin(P.omega * t);
    return Pose{cos(th), sin(th), P.ref_x + P.vx * t, P.ref_y + P.vy * t};
}

// A body has at most 2048 vertices: eight per thread.
constexpr int T_PLAN = 256;
constexpr int PLAN_VPT = 8;

// (value, index) pairs ordered by value, then index: the least pair is the first vertex
// among those with the least value, as a sequential scan with strict comparisons keeps.
__device__ inline void lexmin(double& v, int& k, double v2, int k2) {
    if (v2 < v || (v2 == v && k2 < k)) {
        v = v2;
        k = k2;
    }
}

// Block reductions of F fields through LDS: the first T_PLAN threads store their partials,
// then each wavefront of the block reduces a field at a time (four loads per lane, then six
// exchange rounds), so one exchange per round and field instead of one per round for every
// field.
template <int F>
struct PlanScratch {
    double v[F][T_PLAN];
    int k[F][T_PLAN];
    double rv[F];
    int rk[F];
};
constexpr int PLAN_F = 8;

// Least (value, index) pair of each field; the results in sc.rv / sc.rk for every thread.
template <int F>
__device__ inline void block_lexmin(const double* v, const int* k, PlanScratch<PLAN_F>& sc) {
    if (threadIdx.x < T_PLAN) {
#pragma unroll
        for (int f = 0; f < F; f++) {
            sc.v[f][threadIdx.x] = v[f];
            sc.k[f][threadIdx.x] = k[f];
        }
    }
    __syncthreads();
    int lane = threadIdx.x & 63;
    for (int f = threadIdx.x >> 6; f < F; f += blockDim.x / 64) {
        double bv = sc.v[f][lane];
        int bk = sc.k[f][lane];
        for (int j = lane + 64; j < T_PLAN; j += 64) lexmin(bv, bk, sc.v[f][j], sc.k[f][j]);
        for (int off = 32; off > 0; off >>= 1) lexmin(bv, bk, __shfl_xor(bv, off, 64), __shfl_xor(bk, off, 64));
        if (lane == 0) {
            sc.rv[f] = bv;
            sc.rk[f] = bk;
        }
    }
    __syncthreads();
}
// Sum of each field (any order); the results in sc.rv for every thread.
template <int F>
__device__ inline void block_sum(const double* v, PlanScratch<PLAN_F>& sc) {
    if (threadIdx.x < T_PLAN) {
#pragma unroll
        for (int f = 0; f < F; f++) sc.v[f][threadIdx.x] = v[f];
    }
    __syncthreads();
    int lane = threadIdx.x & 63;
    for (int f = threadIdx.x >> 6; f < F; f += blockDim.x / 64) {
        double bv = sc.v[f][lane];
        for (int j = lane + 64; j < T_PLAN; j += 64) bv += sc.v[f][j];
        for (int off = 32; off > 0; off >>= 1) bv += __shfl_xor(bv, off, 64);
        if (lane == 0) sc.rv[f] = bv;
    }
    __syncthreads();
}

// Copy of n bytes (a multiple of 8) by the whole block.
__device__ inline void block_copy(void* dst, const void* src, size_t n) {
    for (size_t k = threadIdx.x; k < n / 8; k += blockDim.x)
        ((unsigned long long*)dst)[k] = ((const unsigned long long*)src)[k];
}

// The parts of a step's arguments that make it do nothing: no geometry jobs, empty sweep
// boxes, no dense direction.
__device__ inline void null_step(const PlanConst& P, const PlanState& S, StepArgs& a) {
    a.geo[0].active = a.geo[1].active = 0;
    for (int s = 0; s < 2; s++) {
        a.sw[s].B = Box{0, 0, 0, 0};
        a.sw[s].dir = 2;
        a.sw[s].Uin = a.sw[s].Uout = P.u[S.cur];
    }
}

// One step's planning: dt from the speeds the last step left (cfl_out), then the poses,
// regions, boxes and motion of the step, then the bookkeeping of its end (slots swapped,
// clock advanced, direction order reversed); nothing once the run's steps are planned.
// The whole block calls it (at least T_PLAN threads; the first T_PLAN do the vertex work):
// the first step of a run in a launch of its own, every later one at the end of the step
// before it, in the block that combines that step's wave speeds.
__device__ __forceinline__ void plan_block(const PlanConst* PC, PlanState* PS, StepArgs* out, double* dt_log) {
    // everything the block reads more than once is staged in LDS first (one round trip):
    // the planning is a chain of short dependent steps, each of which would otherwise wait
    // for memory
    __shared__ PlanConst P;
    __shared__ PlanState S;
    __shared__ PlanScratch<PLAN_F> sc;
    __shared__ double sdt;
    __shared__ int halt;
    const double* body = PC->body;
    int m = PC->m;
    bool worker = threadIdx.x < T_PLAN;
    double bxv[PLAN_VPT], byv[PLAN_VPT];
#pragma unroll
    for (int r = 0; r < PLAN_VPT; r++) {
        int k = threadIdx.x + r * T_PLAN;
        bxv[r] = worker && k < m ? body[2 * k] : 0.0;
        byv[r] = worker && k < m ? body[2 * k + 1] : 0.0;
    }
    block_copy(&S, PS, sizeof(PlanState));
    __syncthreads();
    if (S.remaining <= 0) return;
    block_copy(&P, PC, sizeof(PlanConst));
    // the constant arguments go out first; the step's own fields are written over them
    block_copy(out, &PC->base, sizeof(StepArgs));
    double sx = __longlong_as_double((long long)PC->base.cfl_out[0]);
    double sy = __longlong_as_double((long long)PC->base.cfl_out[1]);
    __syncthreads();
    if (threadIdx.x == 0) {
        halt = S.halt;
        if (!halt) {
            unsigned int st = __hip_atomic_load(P.base.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (st & (2u | 8u)) halt = HALT_STATUS;  // bit 1 is only reported
        }
        if (!halt && !(isfinite(sx) && isfinite(sy))) halt = HALT_SPEEDS;
    }
    double t0 = S.t;
    bool turning = P.amp != 0.0;
    int lane = threadIdx.x & 63;
    // a turning body's angle terms at t0: those the last planned step left for its end,
    // else computed (sincos per lane, the same value in every lane)
    double s0w = 0.0, c0w = 1.0, cth0 = 1.0, sth0 = 0.0;
    Pose q0;
    if (!turning) {
        q0 = pose_at_dev(P, t0);
    } else {
        if (S.trig_ok && S.trig_t == t0) {
            s0w = S.sin_w;
            c0w = S.cos_w;
            cth0 = S.cs_th;
            sth0 = S.sn_th;
        } else {
            sincos(P.omega * t0, &s0w, &c0w);
            sincos(P.theta0 + P.amp * s0w, &sth0, &cth0);
        }
        q0 = Pose{cth0, sth0, P.ref_x + P.vx * t0, P.ref_y + P.vy * t0};
    }
    auto pose_k = [&](const Pose& px, const Pose& py, int r, double& x, double& y) {
        x = (px.cs * bxv[r] - px.sn * byv[r]) + px.cx;
        y = (py.sn * bxv[r] + py.cs * byv[r]) + py.cy;
    };
    // vertex speeds at t^n: the rigid velocity of each vertex of the posed body (a body
    // that does not turn moves every vertex with v)
    if (m > 0 && !turning) {
        sx = fmax(sx, fabs(P.vx));
        sy = fmax(sy, fabs(P.vy));
    } else if (m > 0) {
        double thd = P.amp * P.omega * c0w;
        double cx = P.ref_x + P.vx * t0, cy = P.ref_y + P.vy * t0;
        double v[2] = {-sx, -sy};  // maxima as least negated values
        int kk[2] = {0, 0};
#pragma unroll
        for (int r = 0; r < PLAN_VPT; r++) {
            if (!worker || (int)threadIdx.x + r * T_PLAN >= m) continue;
            double x, y;
            pose_k(q0, q0, r, x, y);
            double ux = P.vx - thd * (y - cy);
            double uy = P.vy + thd * (x - cx);
            v[0] = fmin(v[0], -fabs(ux));
            v[1] = fmin(v[1], -fabs(uy));
        }
        block_lexmin<2>(v, kk, sc);
        sx = -sc.rv[0];
        sy = -sc.rv[1];
    }
    if (threadIdx.x == 0) {
        double dt = P.cfl * fmin(P.hx / sx, P.hy / sy);
        if (!halt && (!(dt > 0.0) || !isfinite(dt))) halt = HALT_DT;
        sdt = dt;
    }
    __syncthreads();
    double dt = sdt;
    double t1 = t0 + dt;
    // a turning body's angle terms at t1 and for the step's motion, in two rounds of one
    // sincos per lane (lane 0: omega t1, then the pose angle th1; lane 1: omega at mid-step,
    // then th1 - th0), shared across the wavefront
    double s1w = 0.0, c1w = 1.0, cth1 = 1.0, sth1 = 0.0, cmid = 1.0, cosd = 1.0, sind = 0.0;
    Pose q1;
    if (!turning) {
        q1 = pose_at_dev(P, t1);
    } else {
        double sa, ca, sb, cb;
        sincos(lane == 0 ? P.omega * t1 : P.omega * (t0 + 0.5 * dt), &sa, &ca);
        s1w = __shfl(sa, 0, 64);
        c1w = __shfl(ca, 0, 64);
        cmid = __shfl(ca, 1, 64);
        double th0 = P.theta0 + P.amp * s0w, th1 = P.theta0 + P.amp * s1w;
        sincos(lane == 0 ? th1 : th1 - th0, &sb, &cb);
        sth1 = __shfl(sb, 0, 64);
        cth1 = __shfl(cb, 0, 64);
        sind = __shfl(sb, 1, 64);
        cosd = __shfl(cb, 1, 64);
        q1 = Pose{cth1, sth1, P.ref_x + P.vx * t1, P.ref_y + P.vy * t1};
    }
    // stage polygon: the first sweep's coordinate at t^{n+1}, the other at t^n
    Pose mx = S.parity == 0 ? q1 : q0, my = S.parity == 0 ? q0 : q1;
    // per polygon (0: stage, 1: end) the least y, greatest y, least x, greatest x with the
    // first vertex attaining each (greatest values as least negated values)
    double ev[PLAN_F];
    int ek[PLAN_F];
    double sums[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int f = 0; f < PLAN_F; f++) {
        ev[f] = INFINITY;
        ek[f] = 0x7fffffff;
    }
    // a body that does not turn is translated: its extremes follow from the turned body's,
    // and the motion check needs the vertices only when the translation is close to a cell
    bool check = turning || !(surely_within(q0.cx, q1.cx, P.hx, P.ext0.mag) &&
                              surely_within(q0.cy, q1.cy, P.hy, P.ext0.mag));
    int bad = 0;
    if (!halt && m > 0 && check) {
#pragma unroll
        for (int r = 0; r < PLAN_VPT; r++) {
            int k = threadIdx.x + r * T_PLAN;
            if (!worker || k >= m) continue;
            double x0, y0, x1, y1, xm, ym;
            pose_k(q0, q0, r, x0, y0);
            pose_k(q1, q1, r, x1, y1);
            if (!(fabs(x1 - x0) < P.hx) || !(fabs(y1 - y0) < P.hy)) bad = 1;
            if (!turning) continue;
            pose_k(mx, my, r, xm, ym);
            lexmin(ev[0], ek[0], ym, k);
            lexmin(ev[1], ek[1], -ym, k);
            lexmin(ev[2], ek[2], xm, k);
            lexmin(ev[3], ek[3], -xm, k);
            lexmin(ev[4], ek[4], y1, k);
            lexmin(ev[5], ek[5], -y1, k);
            lexmin(ev[6], ek[6], x1, k);
            lexmin(ev[7], ek[7], -x1, k);
            sums[0] += xm;
            sums[1] += ym;
            sums[2] += x1;
            sums[3] += y1;
        }
    }
    bad = __syncthreads_or(bad);
    double ext_v[PLAN_F];
    int ext_k[PLAN_F];
    if (!halt && m > 0 && turning) {
        block_lexmin<PLAN_F>(ev, ek, sc);
#pragma unroll
        for (int f = 0; f < PLAN_F; f++) {
            ext_v[f] = sc.rv[f];
            ext_k[f] = sc.rk[f];
        }
    } else {
        const Extremes& X = P.ext0;
        const Pose* px[2] = {&mx, &q1};
        const Pose* py[2] = {&my, &q1};
#pragma unroll
        for (int q = 0; q < 2; q++) {
            ext_v[4 * q + 0] = X.ylo + py[q]->cy;
            ext_v[4 * q + 1] = -(X.yhi + py[q]->cy);
            ext_v[4 * q + 2] = X.xlo + px[q]->cx;
            ext_v[4 * q + 3] = -(X.xhi + px[q]->cx);
            ext_k[4 * q + 0] = X.ib;
            ext_k[4 * q + 1] = X.it;
            ext_k[4 * q + 2] = X.il;
            ext_k[4 * q + 3] = X.ir;
        }
    }
    double csum[4] = {0.0, 0.0, 0.0, 0.0};
    if (!halt && m > 0 && turning) {
        __syncthreads();
        block_sum<4>(sums, sc);
#pragma unroll
        for (int f = 0; f < 4; f++) csum[f] = sc.rv[f];
    }
    // certificate discs
    Cert cq[2] = {P.cert0, P.cert0};
    if (!halt && m > 0) {
        if (!turning) {
            if (P.cert0.rin2 >= 0.0) {
                cq[0].cx += mx.cx;
                cq[0].cy += my.cy;
                cq[1].cx += q1.cx;
                cq[1].cy += q1.cy;
            }
        } else {
            // both polygons' discs from one pass over the edges
            double cxq[2] = {csum[0] / m, csum[2] / m}, cyq[2] = {csum[1] / m, csum[3] / m};
            cq[0] = cq[1] = Cert{0.0, 0.0, -1.0, 0.0};
            if (m >= 8) {
                // per polygon: least distance to an edge line, least negated squared radius
                double cv[4] = {INFINITY, -0.0, INFINITY, -0.0};
                int ck[4] = {0, 0, 0, 0};
#pragma unroll
                for (int r = 0; r < PLAN_VPT; r++) {
                    int k = threadIdx.x + r * T_PLAN;
                    if (!worker || k >= m) continue;
                    int k1 = k + 1 == m ? 0 : k + 1;
                    double b1x = body[2 * k1], b1y = body[2 * k1 + 1];
#pragma unroll
                    for (int q = 0; q < 2; q++) {
                        const Pose& px = q == 0 ? mx : q1;
                        const Pose& py = q == 0 ? my : q1;
                        double x, y;
                        pose_k(px, py, r, x, y);
                        double x1 = (px.cs * b1x - px.sn * b1y) + px.cx;
                        double y1 = (py.sn * b1x + py.cs * b1y) + py.cy;
                        double ex = x1 - x, ey = y1 - y;
                        double l2 = ex * ex + ey * ey;
                        if (l2 > 0.0) cv[2 * q] = fmin(cv[2 * q], (ex * (cyq[q] - y) - ey * (cxq[q] - x)) / sqrt(l2));
                        double dx = x - cxq[q], dy = y - cyq[q];
                        cv[2 * q + 1] = fmin(cv[2 * q + 1], -(dx * dx + dy * dy));
                    }
                }
                __syncthreads();
                block_lexmin<4>(cv, ck, sc);
                for (int q = 0; q < 2; q++) {
                    double rin = sc.rv[2 * q], rout = sqrt(-sc.rv[2 * q + 1]);
                    if (rin > 1e-7 * rout && isfinite(rin)) {
                        cq[q].cx = cxq[q];
                        cq[q].cy = cyq[q];
                        cq[q].rin2 = (rin * (1.0 - 1e-6)) * (rin * (1.0 - 1e-6));
                        cq[q].rout2 = (rout * (1.0 + 1e-6)) * (rout * (1.0 + 1e-6));
                    }
                }
            }
        }
    }
    // the step's scalars, in three stages: the two polygons and the motion (one thread
    // each), the regions, boxes and checks (one thread), then the argument block written by
    // the whole block (the level records are most of it)
    __shared__ Poly spl[2];
    __shared__ Box scb[2], sreg[2], sB[2];
    __shared__ int slv[6];  // levels copied into: geo 0, geo 1, sweep 0 start/end, sweep 1 start/end
    if (!halt && m > 0 && threadIdx.x < 2) {
        bool q0s = threadIdx.x == 0;  // constant indices keep the arrays in registers
        int q = threadIdx.x;
        Poly Q = S.lev[q == 0 ? S.sm : S.s1].poly;
        Q.m = m;
        Q.ymin = q0s ? ext_v[0] : ext_v[4];
        Q.ymax = -(q0s ? ext_v[1] : ext_v[5]);
        Q.xmin = q0s ? ext_v[2] : ext_v[6];
        Q.xmax = -(q0s ? ext_v[3] : ext_v[7]);
        Q.ib = q0s ? ext_k[0] : ext_k[4];
        Q.it = q0s ? ext_k[1] : ext_k[5];
        Q.il = q0s ? ext_k[2] : ext_k[6];
        Q.ir = q0s ? ext_k[3] : ext_k[7];
        const Cert& C = q0s ? cq[0] : cq[1];
        Q.cx = C.cx;
        Q.cy = C.cy;
        Q.rin2 = C.rin2;
        Q.rout2 = C.rout2;
        spl[q] = Q;
        scb[q] = cells_of_bbox(Q.xmin, Q.xmax, Q.ymin, Q.ymax, P.x_lo, P.x_hi, P.y_lo, P.y_hi, P.hx, P.hy, P.nx, P.ny);
    }
    __shared__ Motion smot;
    if (threadIdx.x == 64) {  // another wavefront: the motion's trigonometry runs beside the boxes
        Motion M = S.mot;
        if (!halt && m > 0) {
            // rigid map of the step and the wall velocity at mid-step
            // a body that does not turn has th1 - th0 = 0 exactly: cos 1, sin 0 (exact values)
            M.cosd = cosd;
            M.sind = sind;
            M.c0x = P.ref_x + P.vx * t0;
            M.c0y = P.ref_y + P.vy * t0;
            M.c1x = P.ref_x + P.vx * t1;
            M.c1y = P.ref_y + P.vy * t1;
            double th = t0 + 0.5 * dt;
            M.vx = P.vx;
            M.vy = P.vy;
            double ct = 1.0;  // cos 0
            if (turning) ct = cmid;
            else if (P.omega != 0.0) ct = cos(P.omega * th);
            M.thd = P.amp * P.omega * ct;
            M.chx = P.ref_x + P.vx * th;
            M.chy = P.ref_y + P.vy * th;
        }
        smot = M;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (!halt && m > 0 && bad) halt = HALT_MOTION;
        if (!halt && m > 0) {
            Box rm = box_union(S.lbox[S.sm], scb[0]), r1 = box_union(S.lbox[S.s1], scb[1]);
            auto fits = [&](const Box& r) { return box_empty(r) || (r.w() <= P.gw && r.h() <= P.gh); };
            if (!fits(rm) || !fits(r1)) {
                halt = HALT_REGION;
            } else {
                S.lev[S.sm].poly = spl[0];
                S.lev[S.s1].poly = spl[1];
                S.lbox[S.sm] = scb[0];
                S.lbox[S.s1] = scb[1];
                sreg[0] = rm;
                sreg[1] = r1;
            }
        }
        if (!halt) {
            S.mot = smot;
            slv[0] = S.sm;
            slv[1] = S.s1;
            slv[2] = S.s0;
            slv[3] = S.sm;
            slv[4] = S.sm;
            slv[5] = S.s1;
            for (int s = 0; s < 2; s++) {
                sB[s] = sweep_box_of(S.lbox[slv[2 + 2 * s]], S.lbox[slv[3 + 2 * s]], P.nx, P.ny);
                if (!box_empty(sB[s]) && (sB[s].w() > P.capw || sB[s].h() > P.caph)) halt = HALT_SWEEP_CAP;
            }
        }
    }
    __syncthreads();
    StepArgs& A = *out;
    if (halt) {
        if (threadIdx.x == 0) {
            null_step(P, S, A);
            S.halt = halt;
        }
    } else {
        // level records: 6 x 16 words, one word per thread
        constexpr int LW = sizeof(Level) / 8;
        if (threadIdx.x < 6 * LW) {
            int r = threadIdx.x / LW, w = threadIdx.x % LW;
            Level* dst = r == 0 ? &A.geo[0].L : r == 1 ? &A.geo[1].L : r == 2 ? &A.sw[0].Ls
                       : r == 3 ? &A.sw[0].Le : r == 4 ? &A.sw[1].Ls : &A.sw[1].Le;
            ((unsigned long long*)dst)[w] = ((const unsigned long long*)&S.lev[slv[r]])[w];
        }
        int tid = (int)threadIdx.x - 6 * LW;
        if (m > 0 && (tid == 0 || tid == 1)) {
            GeoJob& J = A.geo[tid];
            Pose px = tid == 0 ? mx : q1;
            Pose py = tid == 0 ? my : q1;
            J.reg = sreg[tid];
            J.cs_x = px.cs;
            J.sn_x = px.sn;
            J.cx_x = px.cx;
            J.cs_y = py.cs;
            J.sn_y = py.sn;
            J.cy_y = py.cy;
            J.active = !box_empty(sreg[tid]);
        }
        if (tid == 2 || tid == 3) {
            int s = tid - 2;
            SweepJob& J = A.sw[s];
            int first = s == 0;
            J.B = sB[s];
            J.dir = first ? S.parity : 1 - S.parity;
            J.first = first;
            J.lam = dt / (J.dir == 0 ? P.hx : P.hy);
            int rin = first ? S.cur : 1 - S.cur;
            J.Uin = P.u[rin];
            J.Uout = P.u[1 - rin];
        }
        if (tid == 4) {
            A.mot = S.mot;
            A.step_id = (int32_t)(S.step & 0x7fffffff);
        }
    }
    __syncthreads();  // every stage-C reader of S is done
    if (threadIdx.x == 0) S.remaining--;
    if (!halt && threadIdx.x == 0) {
        S.last_sweep_box = sB[1];
        // the step's end: slots swapped, clock advanced, the direction order reversed
        dt_log[S.steps] = dt;
        S.step_dt = dt;
        int tmp = S.s0;
        S.s0 = S.s1;
        S.s1 = tmp;
        S.t = t0 + dt;
        S.trig_ok = turning ? 1 : 0;
        S.trig_t = S.t;
        S.sin_w = s1w;
        S.cos_w = c1w;
        S.cs_th = cth1;
        S.sn_th = sth1;
        S.step++;
        S.parity ^= 1;
        S.steps++;
    }
    __syncthreads();
    block_copy(PS, &S, sizeof(PlanState));
}

__global__ __launch_bounds__(T_PLAN) void kb_plan(const PlanConst* PC, PlanState* PS, StepArgs* out, double* dt_log) {
    plan_block(PC, PS, out, dt_log);
}

}  // namespace cc
