// Cut-cell geometry kernels for one level (Sec. 2.1 volume fractions, Sec. 2.2 face
// apertures, Sec. 2.3.4 time-averaged apertures).  The body is a convex polygon.
//
// Work is restricted to the polygon's bounding box (plus the region the level slot
// occupied before, which is reset to fluid): vertices outside the box are fluid, faces
// outside it are open, cells outside it are regular.
#pragma once
#include "cc_device.h"

namespace cc {

// ------------------------------------------------------------ wave-parallel variants
// One 64-lane wavefront handles one face / cell / vertex; the polygon's edges are split
// across the lanes and combined with exact (order-independent) max/min/any reductions, or
// a fixed xor tree for sums, so the O(m) loops run 64x shorter.
constexpr int WAVE = 64;

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, WAVE));
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Closed-polygon membership: solid iff on or left of every edge (boundary is solid);
// outside the bounding box fluid.  The certificate discs (inscribed / circumscribed about
// (cx, cy), shrunk and grown by a relative 1e-6) decide points whose orientation signs
// cannot be affected by rounding, so the result is that of testing every edge; the
// any-negative vote over the lanes is order-independent.
__device__ __forceinline__ int wave_classify(const Poly& P, double px, double py, int lane) {
    if (P.m == 0) return FLUID;
    if (px < P.xmin || px > P.xmax || py < P.ymin || py > P.ymax) return FLUID;
    if (P.rin2 >= 0.0) {
        double dx = px - P.cx, dy = py - P.cy;
        double d2 = dx * dx + dy * dy;
        if (d2 < P.rin2) return SOLID;
        if (d2 > P.rout2) return FLUID;
    }
    const double* v = P.v;
    int neg = 0;
    for (int k = lane; k < P.m; k += WAVE) {
        int k1 = k + 1 == P.m ? 0 : k + 1;
        if (orient(v[2 * k], v[2 * k + 1], v[2 * k1], v[2 * k1 + 1], px, py) < 0.0) {
            neg = 1;
            break;
        }
    }
    return __any(neg) ? FLUID : SOLID;
}

// Solid parameter interval of the segment A->B (Cyrus-Beck against the half-planes):
// empty if some edge has both end points outside, else [max entering t, min leaving t];
// the max/min over the lanes are exact.
__device__ __forceinline__ double2 wave_seg_clip(const Poly& P, double ax, double ay, double bx, double by,
                                                  int lane) {
    double tl = 0.0, th = 1.0;
    int rej = 0;
    const double* v = P.v;
    for (int k = lane; k < P.m; k += WAVE) {
        int k1 = k + 1 == P.m ? 0 : k + 1;
        double ex = v[2 * k], ey = v[2 * k + 1], fx = v[2 * k1], fy = v[2 * k1 + 1];
        double g0 = orient(ex, ey, fx, fy, ax, ay), g1 = orient(ex, ey, fx, fy, bx, by);
        if (g0 < 0.0 && g1 < 0.0) {
            rej = 1;
            break;
        }
        if (g0 >= 0.0 && g1 >= 0.0) continue;
        double t = g0 / (g0 - g1);
        if (g0 < 0.0) {
            if (t > tl) tl = t;
        } else {
            if (t < th) th = t;
        }
    }
    if (__any(rej)) return make_double2(0.0, 0.0);
    tl = wave_max(tl);
    th = wave_min(th);
    if (!(tl < th)) return make_double2(0.0, 0.0);
    return make_double2(tl, th);
}

__device__ __forceinline__ double2 wave_face_interval(const Poly& P, double ax, double ay, int ca, double bx,
                                                      double by, int cb, int lane) {
    if (P.m == 0) return make_double2(0.0, 0.0);
    if (ca == SOLID && cb == SOLID) return make_double2(0.0, 1.0);
    if (fmax(ax, bx) < P.xmin || fmin(ax, bx) > P.xmax || fmax(ay, by) < P.ymin || fmin(ay, by) > P.ymax)
        return make_double2(0.0, 0.0);
    return wave_seg_clip(P, ax, ay, bx, by, lane);
}

// Solid length of the right side {w} x [0, h] of a rectangle (coordinates relative to its
// corner (ox, oy)).  The boundary of a counter-clockwise convex polygon crosses the line
// x = w going right at its lower crossing and going left at its upper one.  Both crossings
// are computed exactly as the edge clipping computes them (t = (w - ax)/dx,
// y = ay + t dy), so the area's edge sum and this side term use the same points and their
// rounding cancels, also where the line is nearly tangent to the body.
__device__ double wave_right_solid(const Poly& P, double ox, double oy, double w, double h, int lane) {
    double yb = -INFINITY, yt = INFINITY;
    int found = 0;
    const double* v = P.v;
    for (int k = lane; k < P.m; k += WAVE) {
        int k1 = k + 1 == P.m ? 0 : k + 1;
        double ax = v[2 * k] - ox, ay = v[2 * k + 1] - oy;
        double bx = v[2 * k1] - ox, by = v[2 * k1 + 1] - oy;
        if ((ax < w) == (bx < w)) continue;  // half-open straddle rule
        double dx = bx - ax, dy = by - ay;
        double t = (w - ax) / dx;
        double y = ay + t * dy;
        found = 1;
        if (dx > 0.0) yb = fmax(yb, y);
        else yt = fmin(yt, y);
    }
    if (!__any(found)) return 0.0;
    yb = wave_max(yb);
    yt = wave_min(yt);
    double lo = fmax(0.0, yb), hi = fmin(h, yt);
    return hi > lo ? hi - lo : 0.0;
}

// Area of the polygon inside the rectangle [ox, ox+w] x [oy, oy+h] by Green's theorem:
// the integral of x dy over the part of the polygon boundary inside the rectangle (each
// edge clipped with Liang-Barsky in coordinates relative to (ox, oy); the coordinate of a
// clipped end point that lies on a rectangle side is set exactly) plus w times the solid
// length of the rectangle's right side (the bottom, top and left sides contribute nothing).
// The edge sum is split across the lanes and added with a fixed xor tree.
__device__ double wave_clip_area(const Poly& P, double ox, double oy, double w, double h, double right_solid,
                                 int lane) {
    double acc = 0.0;
    const double* v = P.v;
    for (int k = lane; k < P.m; k += WAVE) {
        int k1 = k + 1 == P.m ? 0 : k + 1;
        double ax = v[2 * k] - ox, ay = v[2 * k + 1] - oy;
        double bx = v[2 * k1] - ox, by = v[2 * k1 + 1] - oy;
        if (fmax(ax, bx) < 0.0 || fmin(ax, bx) > w || fmax(ay, by) < 0.0 || fmin(ay, by) > h) continue;
        double dx = bx - ax, dy = by - ay;
        double t0 = 0.0, t1 = 1.0;
        int s0 = -1, s1 = -1;
        double pq[4][2] = {{-dx, ax}, {dx, w - ax}, {-dy, ay}, {dy, h - ay}};
        bool rej = false;
#pragma unroll
        for (int s = 0; s < 4; s++) {
            double p = pq[s][0], q = pq[s][1];
            if (p == 0.0) {
                // parallel to this side: outside, or lying on the right side, whose solid
                // part the right-side term already counts
                if (q < 0.0 || (s == 1 && q == 0.0)) rej = true;
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
    return wave_sum(acc) + w * right_solid;
}

// ---------------------------------------------------------------------------- kernels
// Launch shape of the wave-per-item kernels: 256 threads = 4 items per block.
constexpr int ITEMS_PER_BLOCK = 4;

__device__ __forceinline__ int wave_item() { return blockIdx.x * ITEMS_PER_BLOCK + (threadIdx.x >> 6); }
__device__ __forceinline__ int wave_lane() { return threadIdx.x & 63; }

// Vertex classes over vertices [vi0, vi0+vw) x [vj0, vj0+vh).
__global__ __launch_bounds__(256) void k_geo_vertices(Grid g, Level L, int vi0, int vj0, int vw, int vh) {
    int t = wave_item(), lane = wave_lane();
    if (t >= vw * vh) return;
    int i = vi0 + t % vw, j = vj0 + t / vw;
    int c = wave_classify(L.poly, vx_of(g, i), vy_of(g, j), lane);
    if (lane == 0) L.vcls[(size_t)j * (g.nx + 1) + i] = (int8_t)c;
}

// Face solid intervals.  x-faces: i in [vi0, vi0+vw), j in [vj0, vj0+vh-1);
// y-faces: i in [vi0, vi0+vw-1), j in [vj0, vj0+vh).
__global__ __launch_bounds__(256) void k_geo_faces(Grid g, Level L, int vi0, int vj0, int vw, int vh) {
    int t = wave_item(), lane = wave_lane();
    int nfx = vw * (vh - 1), nfy = (vw - 1) * vh;
    if (t >= nfx + nfy) return;
    const int8_t* vc = L.vcls;
    int W1 = g.nx + 1;
    if (t < nfx) {
        int i = vi0 + t % vw, j = vj0 + t / vw;
        double x = vx_of(g, i);
        double2 iv = wave_face_interval(L.poly, x, vy_of(g, j), vc[(size_t)j * W1 + i], x, vy_of(g, j + 1),
                                        vc[(size_t)(j + 1) * W1 + i], lane);
        if (lane == 0) L.fx[(size_t)j * W1 + i] = iv;
    } else {
        t -= nfx;
        int i = vi0 + t % (vw - 1), j = vj0 + t / (vw - 1);
        double y = vy_of(g, j);
        double2 iv = wave_face_interval(L.poly, vx_of(g, i), y, vc[(size_t)j * W1 + i], vx_of(g, i + 1), y,
                                        vc[(size_t)j * W1 + i + 1], lane);
        if (lane == 0) L.fy[(size_t)j * g.nx + i] = iv;
    }
}

// Volume fractions over cells [ci0, ci0+cw) x [cj0, cj0+ch): open when all four faces are
// open, closed when all four are closed, otherwise 1 - (polygon area in the cell)/(hx hy).
__global__ __launch_bounds__(256) void k_geo_cells(Grid g, Level L, int ci0, int cj0, int cw, int ch) {
    int t = wave_item(), lane = wave_lane();
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
        double ox = vx_of(g, i), oy = vy_of(g, j);
        double rs = wave_right_solid(L.poly, ox, oy, g.hx, g.hy, lane);
        double s = wave_clip_area(L.poly, ox, oy, g.hx, g.hy, rs, lane);
        a = 1.0 - s / (g.hx * g.hy);
        if (a < 0.0) a = 0.0;
        if (a > 1.0) a = 1.0;
        if (a < g.alpha_min) a = 0.0;  // small-cell threshold: counts as solid
    }
    if (lane == 0) L.alpha[(size_t)j * g.nx + i] = a;
}

}  // namespace cc
