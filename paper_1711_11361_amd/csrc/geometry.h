// Cut-cell geometry kernels for one level (Sec. 2.1 volume fractions, Sec. 2.2 face
// apertures, Sec. 2.3.4 time-averaged apertures).  The body is a convex polygon.
//
// Work is restricted to the polygon's bounding box (plus the region the level slot
// occupied before, which is reset to fluid): vertices outside the box are fluid, faces
// outside it are open, cells outside it are regular.
#pragma once
#include "cc_device.h"

namespace cc {

// Closed-polygon membership: solid iff on or left of every edge; outside the bounding box
// fluid.  The certificate discs (inscribed / circumscribed about (cx, cy), shrunk and
// grown by a relative 1e-6) decide points whose orientation signs cannot be affected by
// rounding, so the result is identical to testing every edge.
__device__ __forceinline__ int classify(const Poly& P, double px, double py) {
    if (P.m == 0) return FLUID;
    if (px < P.xmin || px > P.xmax || py < P.ymin || py > P.ymax) return FLUID;
    if (P.rin2 >= 0.0) {
        double dx = px - P.cx, dy = py - P.cy;
        double d2 = dx * dx + dy * dy;
        if (d2 < P.rin2) return SOLID;
        if (d2 > P.rout2) return FLUID;
    }
    const double* v = P.v;
    double ax = v[2 * (P.m - 1)], ay = v[2 * (P.m - 1) + 1];
    // edge k runs from vertex k to k+1; walk them starting with the closing edge
    for (int k = 0; k < P.m; k++) {
        double bx = v[2 * k], by = v[2 * k + 1];
        if (orient(ax, ay, bx, by, px, py) < 0.0) return FLUID;
        ax = bx;
        ay = by;
    }
    return SOLID;
}

// Solid parameter interval of the segment A->B (Cyrus-Beck against the half-planes).
__device__ __forceinline__ double2 seg_clip(const Poly& P, double ax, double ay, double bx, double by) {
    double tl = 0.0, th = 1.0;
    const double* v = P.v;
    for (int k = 0; k < P.m; k++) {
        int k1 = k + 1 == P.m ? 0 : k + 1;
        double ex = v[2 * k], ey = v[2 * k + 1], fx = v[2 * k1], fy = v[2 * k1 + 1];
        double g0 = orient(ex, ey, fx, fy, ax, ay), g1 = orient(ex, ey, fx, fy, bx, by);
        if (g0 < 0.0 && g1 < 0.0) return make_double2(0.0, 0.0);
        if (g0 >= 0.0 && g1 >= 0.0) continue;
        double t = g0 / (g0 - g1);
        if (g0 < 0.0) {
            if (t > tl) tl = t;
        } else {
            if (t < th) th = t;
        }
    }
    if (!(tl < th)) return make_double2(0.0, 0.0);
    return make_double2(tl, th);
}

__device__ __forceinline__ double2 face_interval(const Poly& P, double ax, double ay, int ca, double bx,
                                                 double by, int cb) {
    if (P.m == 0) return make_double2(0.0, 0.0);
    if (ca == SOLID && cb == SOLID) return make_double2(0.0, 1.0);
    if (fmax(ax, bx) < P.xmin || fmin(ax, bx) > P.xmax || fmax(ay, by) < P.ymin || fmin(ay, by) > P.ymax)
        return make_double2(0.0, 0.0);
    return seg_clip(P, ax, ay, bx, by);
}

// Area of the polygon inside the rectangle [ox, ox+w] x [oy, oy+h] by Green's theorem:
// the part of the polygon boundary inside the rectangle (each edge clipped with
// Liang-Barsky, in coordinates relative to (ox, oy)) plus the rectangle's right side,
// whose solid length is given (the bottom, top and left sides contribute nothing to the
// integral of x dy).
__device__ double clip_area(const Poly& P, double ox, double oy, double w, double h, double right_solid) {
    double acc = 0.0;
    const double* v = P.v;
    for (int k = 0; k < P.m; k++) {
        int k1 = k + 1 == P.m ? 0 : k + 1;
        double ax = v[2 * k] - ox, ay = v[2 * k + 1] - oy;
        double bx = v[2 * k1] - ox, by = v[2 * k1 + 1] - oy;
        if (fmax(ax, bx) < 0.0 || fmin(ax, bx) > w || fmax(ay, by) < 0.0 || fmin(ay, by) > h) continue;
        double dx = bx - ax, dy = by - ay;
        double t0 = 0.0, t1 = 1.0;
        int s0 = -1, s1 = -1;  // rectangle side that set t0 / t1
        double pq[4][2] = {{-dx, ax}, {dx, w - ax}, {-dy, ay}, {dy, h - ay}};
        bool rej = false;
#pragma unroll
        for (int s = 0; s < 4; s++) {
            double p = pq[s][0], q = pq[s][1];
            if (p == 0.0) {
                if (q < 0.0) rej = true;
            } else {
                double t = q / p;
                if (p < 0.0) {
                    if (t > t0) {
                        t0 = t;
                        s0 = s;
                    }
                } else {
                    if (t < t1) {
                        t1 = t;
                        s1 = s;
                    }
                }
            }
        }
        if (rej || !(t0 < t1)) continue;
        // clipped end points; the coordinate fixed by the clipping side is set exactly
        double x0 = ax + t0 * dx, y0 = ay + t0 * dy;
        double x1 = ax + t1 * dx, y1 = ay + t1 * dy;
        const double side[4] = {0.0, w, 0.0, h};
        if (s0 >= 0) {
            if (s0 < 2) x0 = side[s0]; else y0 = side[s0];
        }
        if (s1 >= 0) {
            if (s1 < 2) x1 = side[s1]; else y1 = side[s1];
        }
        acc += 0.5 * (x0 + x1) * (y1 - y0);
    }
    return acc + w * right_solid;
}

// ---------------------------------------------------------------------------- kernels
// Vertex classes over vertices [vi0, vi0+vw) x [vj0, vj0+vh).
__global__ void k_geo_vertices(Grid g, Level L, int vi0, int vj0, int vw, int vh) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= vw * vh) return;
    int i = vi0 + t % vw, j = vj0 + t / vw;
    L.vcls[(size_t)j * (g.nx + 1) + i] = (int8_t)classify(L.poly, vx_of(g, i), vy_of(g, j));
}

// Face solid intervals.  x-faces: i in [vi0, vi0+vw), j in [vj0, vj0+vh-1);
// y-faces: i in [vi0, vi0+vw-1), j in [vj0, vj0+vh).
__global__ void k_geo_faces(Grid g, Level L, int vi0, int vj0, int vw, int vh) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int nfx = vw * (vh - 1), nfy = (vw - 1) * vh;
    if (t >= nfx + nfy) return;
    const int8_t* vc = L.vcls;
    int W1 = g.nx + 1;
    if (t < nfx) {
        int i = vi0 + t % vw, j = vj0 + t / vw;
        double x = vx_of(g, i);
        L.fx[(size_t)j * W1 + i] = face_interval(L.poly, x, vy_of(g, j), vc[(size_t)j * W1 + i], x,
                                                 vy_of(g, j + 1), vc[(size_t)(j + 1) * W1 + i]);
    } else {
        t -= nfx;
        int i = vi0 + t % (vw - 1), j = vj0 + t / (vw - 1);
        double y = vy_of(g, j);
        L.fy[(size_t)j * g.nx + i] = face_interval(L.poly, vx_of(g, i), y, vc[(size_t)j * W1 + i],
                                                   vx_of(g, i + 1), y, vc[(size_t)j * W1 + i + 1]);
    }
}

// Volume fractions over cells [ci0, ci0+cw) x [cj0, cj0+ch): open when all four faces are
// open, closed when all four are closed, otherwise 1 - (polygon area in the cell)/(hx hy).
__global__ void k_geo_cells(Grid g, Level L, int ci0, int cj0, int cw, int ch) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cw * ch) return;
    int i = ci0 + t % cw, j = cj0 + t / cw;
    double2 ivE = L.fx[(size_t)j * (g.nx + 1) + i + 1];
    double b[4] = {beta_x(g, L, i, j), interval_beta(ivE), beta_y(g, L, i, j), beta_y(g, L, i, j + 1)};
    int ones = 0, zeros = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        ones += b[k] == 1.0;
        zeros += b[k] == 0.0;
    }
    double a;
    if (ones == 4) {
        a = 1.0;
    } else if (zeros == 4) {
        a = 0.0;
    } else {
        double rs = ivE.y > ivE.x ? (ivE.y - ivE.x) * g.hy : 0.0;
        double s = clip_area(L.poly, vx_of(g, i), vy_of(g, j), g.hx, g.hy, rs);
        a = 1.0 - s / (g.hx * g.hy);
        if (a < 0.0) a = 0.0;
        if (a > 1.0) a = 1.0;
    }
    L.alpha[(size_t)j * g.nx + i] = a;
}

}  // namespace cc
