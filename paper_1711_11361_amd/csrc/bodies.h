// Several bodies in one context (the sloped moving channel of Sec. 3.1, whose two walls
// are two solid regions moving together, and bodies in relative motion after Sec. 3.5).
// The solid region is the union of up to MAX_BODIES closed convex polygons, each posed
// with its own rigid motion.  They must keep apart: a face with solid parts of two bodies,
// a cell with solid area of two bodies, or a wall cell cut by one body at a sweep's start
// and by another at its end sets status bit 4.  Per level:
//   vertex class: solid when inside (or on) any body;
//   face interval: the solid interval of the one body that meets the face in a segment of
//     positive length (ends classified against that body);
//   volume fraction: 1 - (sum of the bodies' areas in the cell) / (hx hy) for cut cells;
//   body of a cut cell: the first body with area in the cell, else the first that closes
//     part of one of its faces, else body 0.
// Per sweep, the exact time-averaged aperture of a face across the sweep direction sums
// the bodies' swept areas, each over the strip its own displacement sweeps; a body that
// does not move there contributes the mean of its solid fractions of the face at the
// sweep's two levels.  Every item is done by one thread with the plain edge loops (the
// bodies of such scenes have few edges).
#pragma once
#include "sweep.h"

namespace cc {

__device__ __forceinline__ int body_class(const Poly& P, double px, double py) {
    int c = classify_quick(P, px, py);
    return c >= 0 ? c : poly_classify<1>(P, px, py, 0);
}

// Solid interval of segment A->B against one body (its own classes of the ends).
__device__ __forceinline__ double2 body_face(const Poly& P, double ax, double ay, double bx, double by) {
    int ca = body_class(P, ax, ay), cb = body_class(P, bx, by);
    double2 iv;
    if (!face_quick(P, ax, ay, ca, bx, by, cb, iv)) iv = poly_seg_clip<1>(P, ax, ay, bx, by, 0);
    return iv;
}

__device__ __forceinline__ double body_face_solid(const Poly& P, double ax, double ay, double bx, double by) {
    double2 iv = body_face(P, ax, ay, bx, by);
    return iv.y > iv.x ? iv.y - iv.x : 0.0;
}

// Closed bounding boxes of the body and of [x0, x1] x [y0, y1] are disjoint.
__device__ __forceinline__ bool body_misses(const Poly& P, double x0, double y0, double x1, double y1) {
    return P.m == 0 || x1 < P.xmin || x0 > P.xmax || y1 < P.ymin || y0 > P.ymax;
}

// Body of cut cell (i, j) that covers no area of it: the first that closes part of one of
// its faces (W, E, S, N), else 0.
__device__ int cell_touching_body(const Grid& g, const Level& L, int i, int j) {
    double x0 = vx_of(g, i), x1 = vx_of(g, i + 1), y0 = vy_of(g, j), y1 = vy_of(g, j + 1);
    const double seg[4][4] = {{x0, y0, x0, y1}, {x1, y0, x1, y1}, {x0, y0, x1, y0}, {x0, y1, x1, y1}};
    for (int b = 0; b < L.np; b++)
        for (int e = 0; e < 4; e++) {
            double2 iv = body_face(L.parts[b], seg[e][0], seg[e][1], seg[e][2], seg[e][3]);
            if (iv.y > iv.x) return b;
        }
    return 0;
}

// Stage K of level job J (0: vertex classes, 1: face intervals, 2: volume fractions and
// cell bodies) with several bodies, block lb of the job's nb.
template <int K>
__device__ void geo_bodies_block(const Grid& g, const GeoJob& J, int lb, int nb, unsigned int* status) {
    const Level& L = J.L;
    int items = K == 0 ? geo_nverts(J.reg) : (K == 1 ? geo_nfaces(J.reg) : J.reg.w() * J.reg.h());
    bool bad = false;
    for (int t = lb * (int)blockDim.x + (int)threadIdx.x; t < items; t += nb * (int)blockDim.x) {
        if (K == 0) {
            int vw = J.reg.w() + 1;
            int i = J.reg.i0 + t % vw, j = J.reg.j0 + t / vw;
            double px = vx_of(g, i), py = vy_of(g, j);
            int c = FLUID;
            for (int b = 0; b < L.np && c == FLUID; b++) c = body_class(L.parts[b], px, py);
            L.vcls[(size_t)j * (g.nx + 1) + i] = (int8_t)c;
        } else if (K == 1) {
            bool xf;
            int i, j, ca, cb;
            double ax, ay, bx, by;
            geo_face_ends(g, J, t, xf, i, j, ax, ay, ca, bx, by, cb);
            double2 iv = make_double2(0.0, 0.0);
            int hits = 0;
            for (int b = 0; b < L.np; b++) {
                double2 q = body_face(L.parts[b], ax, ay, bx, by);
                if (q.y > q.x) {
                    if (hits == 0) iv = q;
                    hits++;
                }
            }
            bad |= hits > 1;
            geo_store_face(g, J, xf, i, j, iv);
        } else {
            int cw = J.reg.w();
            int i = J.reg.i0 + t % cw, j = J.reg.j0 + t / cw;
            double bf[4] = {beta_x(g, L, i, j), beta_x(g, L, i + 1, j), beta_y(g, L, i, j), beta_y(g, L, i, j + 1)};
            int ones = 0, zeros = 0;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                ones += bf[k] == 1.0;
                zeros += bf[k] == 0.0;
            }
            double a;
            int body = -1;
            if (ones == 4) {
                a = 1.0;
            } else if (zeros == 4) {
                a = 0.0;
            } else {
                double x0 = vx_of(g, i), y0 = vy_of(g, j);
                double s = 0.0;
                int hits = 0;
                for (int b = 0; b < L.np; b++) {
                    const Poly& P = L.parts[b];
                    double ab = 0.0;
                    if (!body_misses(P, x0, y0, x0 + g.hx, y0 + g.hy)) ab = poly_clip_area<1>(P, x0, y0, g.hx, g.hy, 0);
                    if (ab > 0.0) {
                        if (hits == 0) body = b;
                        hits++;
                    }
                    s += ab;
                }
                bad |= hits > 1;
                if (body < 0) body = cell_touching_body(g, L, i, j);
                a = alpha_of_area(g, s);
            }
            size_t k = (size_t)j * g.nx + i;
            L.alpha[k] = a;
            L.cbody[k] = (int8_t)body;
        }
    }
    if (bad) atomicOr(status, 4u);
}

// Time-averaged aperture of face t of the sweep box (faces across the sweep direction)
// with several bodies; bm: the bodies' motions of the step.
template <int D>
__device__ void swept_bodies(const Grid& g, const SweepJob& J, const Motion* bm, const Stage& S, int t) {
    const Box& B = J.B;
    int fw = D == 0 ? B.w() + 1 : B.w(), fh = D == 0 ? B.h() : B.h() + 1;
    if (t >= fw * fh) return;
    int i = B.i0 + t % fw, j = B.j0 + t / fw;
    double bs = D == 0 ? beta_x(g, J.Ls, i, j) : beta_y(g, J.Ls, i, j);
    double be = D == 0 ? beta_x(g, J.Le, i, j) : beta_y(g, J.Le, i, j);
    double r = 0.0;  // covered throughout (the bodies keep apart)
    if (!(bs == 0.0 && be == 0.0)) {
        double X = vx_of(g, i), Y = vy_of(g, j);
        double h = D == 0 ? g.hx : g.hy, hf = D == 0 ? g.hy : g.hx;
        double fx = D == 0 ? X : X + g.hx, fy = D == 0 ? Y + g.hy : Y;
        double solid = 0.0;
        for (int b = 0; b < J.Ls.np; b++) {
            const Poly& Ps = J.Ls.parts[b];
            double Dd = D == 0 ? step_disp(bm[b], 0, X, Y + 0.5 * g.hy) : step_disp(bm[b], 1, X + 0.5 * g.hx, Y);
            if (!(fabs(Dd) > 1e-12 * h)) {
                solid += 0.5 * (body_face_solid(Ps, X, Y, fx, fy) + body_face_solid(J.Le.parts[b], X, Y, fx, fy));
                continue;
            }
            double w = fabs(Dd);
            double x0, y0, sw, sh;
            if (D == 0) {
                x0 = Dd > 0.0 ? X - Dd : X;
                y0 = Y;
                sw = w;
                sh = hf;
            } else {
                x0 = X;
                y0 = Dd > 0.0 ? Y - Dd : Y;
                sw = hf;
                sh = w;
            }
            if (body_misses(Ps, x0, y0, x0 + sw, y0 + sh)) continue;
            solid += poly_clip_area<1>(Ps, x0, y0, sw, sh, 0) / (w * hf);
        }
        r = 1.0 - solid;
        if (r < 0.0) r = 0.0;
        if (r > 1.0) r = 1.0;
    }
    S.bt[fidx<D>(B, i, j)] = r;
}

}  // namespace cc
