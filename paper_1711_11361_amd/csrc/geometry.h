// Cut-cell geometry of one level (Sec. 2.1 volume fractions, Sec. 2.2 face apertures) and
// the polygon clipping used by the exact time-averaged apertures (Sec. 2.3.4).  The body is
// a convex polygon.
//
// One thread per item (vertex, face, cell) settles it when a cheap exact test suffices:
// outside the polygon's bounding box, inside the inscribed or outside the circumscribed
// certificate disc, both face end points solid, all four cell faces open or closed.
// Otherwise a polygon of a few edges is tested edge by edge by the same thread.  For a
// many-sided polygon the item goes to its thread's wavefront: faces and areas find the few
// edges that can matter on the polygon's monotone chains (a 64-way search) and share them
// across the lanes; vertex classes left undecided are walked over all edges.  All paths
// evaluate the same per-edge formulas; only the order of the area sum differs, and it is
// fixed per polygon size.
#pragma once
#include "cc_device.h"

namespace cc {

constexpr int WAVE = 64;
constexpr int SMALL_POLY = 16;  // polygons with at most this many edges are done per thread

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

// Reductions over the lanes that share an item: a whole wavefront (S = WAVE) or the
// thread alone (S = 1).
template <int S>
__device__ __forceinline__ double red_max(double v) {
    if constexpr (S == 1) return v; else return wave_max(v);
}
template <int S>
__device__ __forceinline__ double red_min(double v) {
    if constexpr (S == 1) return v; else return wave_min(v);
}
template <int S>
__device__ __forceinline__ double red_sum(double v) {
    if constexpr (S == 1) return v; else return wave_sum(v);
}
template <int S>
__device__ __forceinline__ bool red_any(bool v) {
    if constexpr (S == 1) return v; else return __any(v);
}

// ------------------------------------------------------------------ certificate discs
// The posed polygon lies inside the disc of squared radius rout2 about (cx, cy) and
// contains the disc of squared radius rin2 (both widened by a relative 1e-6, so that
// rounding cannot turn a test around); rin2 < 0: no discs.
__device__ __forceinline__ bool seg_outside_disc(const Poly& P, double ax, double ay, double bx, double by) {
    if (P.rin2 < 0.0) return false;
    double dx = bx - ax, dy = by - ay;
    double l2 = dx * dx + dy * dy;
    double t = l2 > 0.0 ? ((P.cx - ax) * dx + (P.cy - ay) * dy) / l2 : 0.0;
    t = fmin(fmax(t, 0.0), 1.0);
    double ex = ax + t * dx - P.cx, ey = ay + t * dy - P.cy;
    return ex * ex + ey * ey > P.rout2;
}
__device__ __forceinline__ bool rect_outside_disc(const Poly& P, double x0, double y0, double w, double h) {
    if (P.rin2 < 0.0) return false;
    double ex = fmin(fmax(P.cx, x0), x0 + w) - P.cx, ey = fmin(fmax(P.cy, y0), y0 + h) - P.cy;
    return ex * ex + ey * ey > P.rout2;
}

// ------------------------------------------------------------------ per-item tests
// Closed-polygon membership: solid iff on or left of every edge (boundary is solid).  The
// any-negative vote over the edges is order-independent.
template <int S>
__device__ __forceinline__ int poly_classify(const Poly& P, double px, double py, int lane) {
    const double* v = P.v;
    int neg = 0;
    for (int k = lane; k < P.m; k += S) {
        int k1 = k + 1 == P.m ? 0 : k + 1;
        if (orient(v[2 * k], v[2 * k + 1], v[2 * k1], v[2 * k1 + 1], px, py) < 0.0) {
            neg = 1;
            break;
        }
    }
    return red_any<S>(neg) ? FLUID : SOLID;
}

// Decided without the edge loop, or -1.
__device__ __forceinline__ int classify_quick(const Poly& P, double px, double py) {
    if (P.m == 0) return FLUID;
    if (px < P.xmin || px > P.xmax || py < P.ymin || py > P.ymax) return FLUID;
    if (P.rin2 >= 0.0) {
        double dx = px - P.cx, dy = py - P.cy;
        double d2 = dx * dx + dy * dy;
        if (d2 < P.rin2) return SOLID;
        if (d2 > P.rout2) return FLUID;
    }
    return -1;
}

// Solid parameter interval of the segment A->B (Cyrus-Beck against the half-planes):
// empty if some edge has both end points outside, else [max entering t, min leaving t].
template <int S>
__device__ __forceinline__ double2 poly_seg_clip(const Poly& P, double ax, double ay, double bx, double by,
                                                  int lane) {
    double tl = 0.0, th = 1.0;
    int rej = 0;
    const double* v = P.v;
    for (int k = lane; k < P.m; k += S) {
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
    if (red_any<S>(rej)) return make_double2(0.0, 0.0);
    tl = red_max<S>(tl);
    th = red_min<S>(th);
    if (!(tl < th)) return make_double2(0.0, 0.0);
    return make_double2(tl, th);
}

// Solid interval of a face decided without the edge loop: 1 = set, 0 = needs the loop.
__device__ __forceinline__ int face_quick(const Poly& P, double ax, double ay, int ca, double bx, double by,
                                          int cb, double2& iv) {
    if (P.m == 0) {
        iv = make_double2(0.0, 0.0);
        return 1;
    }
    if (ca == SOLID && cb == SOLID) {  // convex body: the whole segment is solid
        iv = make_double2(0.0, 1.0);
        return 1;
    }
    if (fmax(ax, bx) < P.xmin || fmin(ax, bx) > P.xmax || fmax(ay, by) < P.ymin || fmin(ay, by) > P.ymax ||
        seg_outside_disc(P, ax, ay, bx, by)) {
        iv = make_double2(0.0, 0.0);
        return 1;
    }
    return 0;
}

// Solid length of the right side {w} x [0, h] of a rectangle (coordinates relative to its
// corner (ox, oy)).  The boundary of a counter-clockwise convex polygon crosses the line
// x = w going right at its lower crossing and going left at its upper one.  Both crossings
// are computed exactly as the edge clipping computes them (t = (w - ax)/dx,
// y = ay + t dy), so the area's edge sum and this side term use the same points and their
// rounding cancels, also where the line is nearly tangent to the body.
template <int S>
__device__ double poly_right_solid(const Poly& P, double ox, double oy, double w, double h, int lane) {
    double yb = -INFINITY, yt = INFINITY;
    int found = 0;
    const double* v = P.v;
    for (int k = lane; k < P.m; k += S) {
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
    if (!red_any<S>(found)) return 0.0;
    yb = red_max<S>(yb);
    yt = red_min<S>(yt);
    double lo = fmax(0.0, yb), hi = fmin(h, yt);
    return hi > lo ? hi - lo : 0.0;
}

// Contribution of edge (a, b) (coordinates relative to the rectangle's corner) to the
// integral of x dy over the part of the polygon boundary inside the rectangle [0, w] x
// [0, h]: the edge clipped with Liang-Barsky, a clipped end point that lies on a rectangle
// side set exactly to that side; 0 for an edge outside (or lying on the right side, which
// the side term covers).
__device__ __forceinline__ double edge_area(double ax, double ay, double bx, double by, double w, double h) {
    if (fmax(ax, bx) < 0.0 || fmin(ax, bx) > w || fmax(ay, by) < 0.0 || fmin(ay, by) > h) return 0.0;
    double dx = bx - ax, dy = by - ay;
    double t0 = 0.0, t1 = 1.0;
    int s0 = -1, s1 = -1;
    double pq[4][2] = {{-dx, ax}, {dx, w - ax}, {-dy, ay}, {dy, h - ay}};
    bool rej = false;
#pragma unroll
    for (int s = 0; s < 4; s++) {
        double p = pq[s][0], q = pq[s][1];
        if (p == 0.0) {
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
    if (rej || !(t0 < t1)) return 0.0;
    double x0 = ax + t0 * dx, y0 = ay + t0 * dy;
    double x1 = ax + t1 * dx, y1 = ay + t1 * dy;
    const double side[4] = {0.0, w, 0.0, h};
    if (s0 >= 0) {
        if (s0 < 2) x0 = side[s0]; else y0 = side[s0];
    }
    if (s1 >= 0) {
        if (s1 < 2) x1 = side[s1]; else y1 = side[s1];
    }
    return 0.5 * (x0 + x1) * (y1 - y0);
}

// Area of the polygon inside the rectangle [ox, ox+w] x [oy, oy+h] by Green's theorem:
// the integral of x dy over the part of the polygon boundary inside the rectangle (each
// edge clipped with Liang-Barsky in coordinates relative to (ox, oy); the coordinate of a
// clipped end point that lies on a rectangle side is set exactly) plus w times the solid
// length of the rectangle's right side (the bottom, top and left sides contribute nothing;
// an edge lying on the right side is left to that term).
template <int S>
__device__ double poly_clip_area(const Poly& P, double ox, double oy, double w, double h, int lane) {
    double right_solid = poly_right_solid<S>(P, ox, oy, w, h, lane);
    double acc = 0.0;
    const double* v = P.v;
    for (int k = lane; k < P.m; k += S) {
        int k1 = k + 1 == P.m ? 0 : k + 1;
        acc += edge_area(v[2 * k] - ox, v[2 * k + 1] - oy, v[2 * k1] - ox, v[2 * k1 + 1] - oy, w, h);
    }
    return red_sum<S>(acc) + w * right_solid;
}

// ------------------------------------------------------------------ chains of a polygon
// Position p of the chain that starts at vertex a: vertex (a + p) mod m.
__device__ __forceinline__ int chain_vertex(const Poly& P, int a, int p) {
    int k = a + p;
    return k >= P.m ? k - P.m : k;
}
__device__ __forceinline__ int chain_edges(const Poly& P, int a, int b) {
    int d = b - a;
    return d < 0 ? d + P.m : d;
}
// First position q in [0, len] of the chain from vertex a at which pred(vertex) holds, for
// a predicate that is false and then true along the chain; len + 1 when it never holds.
// The G lanes of a lane group (G = 64: the whole wavefront; 32 or 16: searches of different
// chains or predicates side by side in one wavefront) test G positions per round and
// narrow the range to the gap between the last false and the first true one (two or three
// rounds for 64 lanes and up to 4096 vertices).  Every lane of the group calls it with the
// same arguments; the answer does not depend on G.
template <int G = WAVE, class F>
__device__ __forceinline__ int chain_first(const Poly& P, int a, int len, int lane, F&& pred) {
    int gl = lane & (G - 1), gb = lane & (WAVE - G);  // lane within the group, group's first lane
    int lo = 0, hi = len + 1;  // the answer lies in [lo, hi]; hi stands for "true"
    while (lo < hi) {
        int span = hi - lo;
        int step = (span + G - 1) / G;
        int p = lo + gl * step;
        bool t = p < hi && pred(chain_vertex(P, a, p));
        unsigned long long mask = __ballot(t) >> gb;
        if (G < WAVE) mask &= (1ull << (G & (WAVE - 1))) - 1ull;
        int tested = (span - 1) / step;  // highest lane with a position below hi
        if (mask == 0ull) {
            lo = lo + tested * step + 1;
        } else {
            int f = __ffsll((long long)mask) - 1;
            int pf = lo + f * step;
            lo = f == 0 ? lo : lo + (f - 1) * step + 1;
            hi = pf;
        }
    }
    return lo;
}

// poly_clip_area of a many-sided polygon by one wavefront: only the edges whose y-range
// meets the rectangle's can contribute to the edge integral (the others give exactly 0),
// and on each y-monotone chain they form one run, found by the same tests; the lanes
// share the run's edges.  The right side's crossings are the one sign change of x < w on
// each x-monotone chain.  Every lane calls it; all get the area.
__device__ double poly_clip_area_chains(const Poly& P, double ox, double oy, double w, double h, int lane) {
    const double* v = P.v;
    auto X = [&](int k) { return v[2 * k] - ox; };
    auto Y = [&](int k) { return v[2 * k + 1] - oy; };
    // right side: lower chain il -> ir (x rising), upper chain ir -> il (x falling); the two
    // searches run side by side in the two halves of the wavefront
    double yb = -INFINITY, yt = INFINITY;
    int found = 0;
    int qx;
    {
        int chain = lane >> 5;
        int a = chain == 0 ? P.il : P.ir, b = chain == 0 ? P.ir : P.il;
        qx = chain_first<32>(P, a, chain_edges(P, a, b), lane,
                             [&](int k) { return chain == 0 ? !(X(k) < w) : X(k) < w; });
    }
    int qxs[2] = {__shfl(qx, 0, WAVE), __shfl(qx, 32, WAVE)};
    for (int chain = 0; chain < 2; chain++) {
        int a = chain == 0 ? P.il : P.ir, b = chain == 0 ? P.ir : P.il;
        int len = chain_edges(P, a, b);
        int q = qxs[chain];
        if (q > 0 && q <= len) {
            int k = chain_vertex(P, a, q - 1), k1 = chain_vertex(P, a, q);
            double ax = X(k), ay = Y(k), dx = X(k1) - ax, dy = Y(k1) - ay;
            double t = (w - ax) / dx;
            double y = ay + t * dy;
            found = 1;
            if (dx > 0.0) yb = fmax(yb, y);
            else yt = fmin(yt, y);
        }
    }
    double right_solid = 0.0;
    if (found) {
        double lo = fmax(0.0, yb), hi = fmin(h, yt);
        right_solid = hi > lo ? hi - lo : 0.0;
    }
    double acc = 0.0;
    // right chain ib -> it (y rising): from the first edge whose end reaches y >= 0 to the
    // last whose start has y <= h; left chain it -> ib (y falling): from the first edge whose
    // end has y <= h to the last whose start has y >= 0.  The four searches (two per chain)
    // run side by side in the four quarters of the wavefront.
    int qy;
    {
        int chain = lane >> 5, second = (lane >> 4) & 1;
        int a = chain == 0 ? P.ib : P.it, b = chain == 0 ? P.it : P.ib;
        qy = chain_first<16>(P, a, chain_edges(P, a, b), lane, [&](int k) {
            return second == 0 ? (chain == 0 ? !(Y(k) < 0.0) : !(Y(k) > h)) : (chain == 0 ? Y(k) > h : Y(k) < 0.0);
        });
    }
    int qys[4] = {__shfl(qy, 0, WAVE), __shfl(qy, 16, WAVE), __shfl(qy, 32, WAVE), __shfl(qy, 48, WAVE)};
    for (int chain = 0; chain < 2; chain++) {
        int a = chain == 0 ? P.ib : P.it, b = chain == 0 ? P.it : P.ib;
        int len = chain_edges(P, a, b);
        int q0 = qys[2 * chain], q1 = qys[2 * chain + 1];
        int p0 = q0 > 0 ? q0 - 1 : 0, p1 = q1 - 1 < len - 1 ? q1 - 1 : len - 1;
        for (int p = p0 + lane; p <= p1; p += WAVE) {
            int k = chain_vertex(P, a, p), k1 = chain_vertex(P, a, p + 1);
            acc += edge_area(X(k), Y(k), X(k1), Y(k1), w, h);
        }
    }
    return red_sum<WAVE>(acc) + w * right_solid;
}

// poly_seg_clip of a many-sided polygon and an axis-aligned segment (a face) by one
// wavefront: the binding edges are those where the segment's line crosses the boundary
// (the sign change of the coordinate test on each monotone chain) and their neighbours;
// when the line meets no chain there (it touches the polygon's extreme side), the full
// edge loop decides.  Every lane calls it; all get the interval.
__device__ double2 poly_seg_clip_chains(const Poly& P, double ax, double ay, double bx, double by, int lane) {
    const double* v = P.v;
    bool vertical = ax == bx;  // x-face: the line x = ax; y-face: the line y = ay
    double c = vertical ? ax : ay;
    int cand[2] = {-1, -1};
    for (int chain = 0; chain < 2; chain++) {
        int a, b;
        if (vertical) {
            a = chain == 0 ? P.il : P.ir;
            b = chain == 0 ? P.ir : P.il;
        } else {
            a = chain == 0 ? P.ib : P.it;
            b = chain == 0 ? P.it : P.ib;
        }
        int len = chain_edges(P, a, b);
        int q = chain_first(P, a, len, lane, [&](int k) {
            bool below = (vertical ? v[2 * k] : v[2 * k + 1]) < c;
            return chain == 0 ? !below : below;
        });
        if (q > 0 && q <= len) cand[chain] = chain_vertex(P, a, q - 1);
    }
    if (cand[0] < 0 && cand[1] < 0) return poly_seg_clip<WAVE>(P, ax, ay, bx, by, lane);
    // lanes 0-2: the crossing edge of the first chain and its neighbours; lanes 3-5: the second
    double tl = 0.0, th = 1.0;
    int rej = 0;
    if (lane < 6 && cand[lane / 3] >= 0) {
        int k = cand[lane / 3] + (lane % 3) - 1;
        k = k < 0 ? k + P.m : (k >= P.m ? k - P.m : k);
        int k1 = k + 1 == P.m ? 0 : k + 1;
        double ex = v[2 * k], ey = v[2 * k + 1], fx = v[2 * k1], fy = v[2 * k1 + 1];
        double g0 = orient(ex, ey, fx, fy, ax, ay), g1 = orient(ex, ey, fx, fy, bx, by);
        if (g0 < 0.0 && g1 < 0.0) {
            rej = 1;
        } else if (!(g0 >= 0.0 && g1 >= 0.0)) {
            double t = g0 / (g0 - g1);
            if (g0 < 0.0) tl = t;
            else th = t;
        }
    }
    if (red_any<WAVE>(rej)) return make_double2(0.0, 0.0);
    tl = red_max<WAVE>(tl);
    th = red_min<WAVE>(th);
    if (!(tl < th)) return make_double2(0.0, 0.0);
    return make_double2(tl, th);
}

// ------------------------------------------------------------------ one thread per item
// The chain searches above done by one thread (bisection) instead of a wavefront, for a
// polygon whose four chains are monotone in its stored coordinates (chains_monotone).  A
// predicate that is false and then true along such a chain has one first true position,
// which every search finds, so each item is given the edges the wavefront search gives it.

// First position q in [0, len] of the chain from vertex a at which pred holds, len + 1 when
// it never holds (pred false and then true along the chain).
template <class F>
__device__ __forceinline__ int chain_first_seq(const Poly& P, int a, int len, F&& pred) {
    int lo = 0, hi = len + 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (pred(chain_vertex(P, a, mid))) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// True when y never decreases from ib to it nor increases from it back to ib, and x never
// decreases from il to ir nor increases from ir back to il, in the stored coordinates (a
// posed convex polygon can lose this by rounding where neighbouring vertices are almost
// level).  Every thread of the block calls it.
__device__ __forceinline__ bool chains_monotone(const Poly& P) {
    const double* v = P.v;
    int ly = chain_edges(P, P.ib, P.it), lx = chain_edges(P, P.il, P.ir);
    int bad = 0;
    for (int k = threadIdx.x; k < P.m; k += blockDim.x) {
        int k1 = k + 1 == P.m ? 0 : k + 1;
        int qy = k - P.ib, qx = k - P.il;
        qy += qy < 0 ? P.m : 0;
        qx += qx < 0 ? P.m : 0;
        double y0 = v[2 * k + 1], y1 = v[2 * k1 + 1], x0 = v[2 * k], x1 = v[2 * k1];
        bool oky = qy < ly ? y1 >= y0 : y1 <= y0;
        bool okx = qx < lx ? x1 >= x0 : x1 <= x0;
        bad |= !(oky && okx);
    }
    return !__syncthreads_or(bad);
}

// poly_clip_area_chains by one thread: the same crossings and runs of edges; the edge
// contributions are summed in chain order.
__device__ double poly_clip_area_chains_t(const Poly& P, double ox, double oy, double w, double h) {
    const double* v = P.v;
    auto X = [&](int k) { return v[2 * k] - ox; };
    auto Y = [&](int k) { return v[2 * k + 1] - oy; };
    double yb = -INFINITY, yt = INFINITY;
    int found = 0;
    for (int chain = 0; chain < 2; chain++) {
        int a = chain == 0 ? P.il : P.ir, b = chain == 0 ? P.ir : P.il;
        int len = chain_edges(P, a, b);
        int q = chain_first_seq(P, a, len, [&](int k) { return chain == 0 ? !(X(k) < w) : X(k) < w; });
        if (q > 0 && q <= len) {
            int k = chain_vertex(P, a, q - 1), k1 = chain_vertex(P, a, q);
            double ax = X(k), ay = Y(k), dx = X(k1) - ax, dy = Y(k1) - ay;
            double t = (w - ax) / dx;
            double y = ay + t * dy;
            found = 1;
            if (dx > 0.0) yb = fmax(yb, y);
            else yt = fmin(yt, y);
        }
    }
    double right_solid = 0.0;
    if (found) {
        double lo = fmax(0.0, yb), hi = fmin(h, yt);
        right_solid = hi > lo ? hi - lo : 0.0;
    }
    double acc = 0.0;
    for (int chain = 0; chain < 2; chain++) {
        int a = chain == 0 ? P.ib : P.it, b = chain == 0 ? P.it : P.ib;
        int len = chain_edges(P, a, b);
        int q0 = chain_first_seq(P, a, len, [&](int k) { return chain == 0 ? !(Y(k) < 0.0) : !(Y(k) > h); });
        int q1 = chain_first_seq(P, a, len, [&](int k) { return chain == 0 ? Y(k) > h : Y(k) < 0.0; });
        int p0 = q0 > 0 ? q0 - 1 : 0, p1 = q1 - 1 < len - 1 ? q1 - 1 : len - 1;
        for (int p = p0; p <= p1; p++) {
            int k = chain_vertex(P, a, p), k1 = chain_vertex(P, a, p + 1);
            acc += edge_area(X(k), Y(k), X(k1), Y(k1), w, h);
        }
    }
    return acc + w * right_solid;
}

// poly_seg_clip_chains by one thread: the same candidate edges, and the full edge loop
// when the segment's line meets no chain crossing.
__device__ double2 poly_seg_clip_chains_t(const Poly& P, double ax, double ay, double bx, double by) {
    const double* v = P.v;
    bool vertical = ax == bx;
    double c = vertical ? ax : ay;
    int cand[2] = {-1, -1};
    for (int chain = 0; chain < 2; chain++) {
        int a, b;
        if (vertical) {
            a = chain == 0 ? P.il : P.ir;
            b = chain == 0 ? P.ir : P.il;
        } else {
            a = chain == 0 ? P.ib : P.it;
            b = chain == 0 ? P.it : P.ib;
        }
        int len = chain_edges(P, a, b);
        int q = chain_first_seq(P, a, len, [&](int k) {
            bool below = (vertical ? v[2 * k] : v[2 * k + 1]) < c;
            return chain == 0 ? !below : below;
        });
        if (q > 0 && q <= len) cand[chain] = chain_vertex(P, a, q - 1);
    }
    if (cand[0] < 0 && cand[1] < 0) return poly_seg_clip<1>(P, ax, ay, bx, by, 0);
    double tl = 0.0, th = 1.0;
    for (int e = 0; e < 6; e++) {
        if (cand[e / 3] < 0) continue;
        int k = cand[e / 3] + (e % 3) - 1;
        k = k < 0 ? k + P.m : (k >= P.m ? k - P.m : k);
        int k1 = k + 1 == P.m ? 0 : k + 1;
        double ex = v[2 * k], ey = v[2 * k + 1], fx = v[2 * k1], fy = v[2 * k1 + 1];
        double g0 = orient(ex, ey, fx, fy, ax, ay), g1 = orient(ex, ey, fx, fy, bx, by);
        if (g0 < 0.0 && g1 < 0.0) return make_double2(0.0, 0.0);
        if (g0 >= 0.0 && g1 >= 0.0) continue;
        double t = g0 / (g0 - g1);
        if (g0 < 0.0) tl = fmax(tl, t);
        else th = fmin(th, t);
    }
    if (!(tl < th)) return make_double2(0.0, 0.0);
    return make_double2(tl, th);
}

// ------------------------------------------------------------------ one level
// Geometry job of one level: the destination slot and the cell region recomputed (its
// vertices and faces are those of the region's closure).  The vertices are posed on the
// device: x from one rigid pose, y from another (the stage polygon of a split step mixes
// the poses at the step's start and end), with the host's formula and operation order.
struct GeoJob {
    Level L;
    Box reg;
    const double* body;             // body-frame vertices (2 m)
    double cs_x, sn_x, cx_x;        // pose giving the x coordinates: cs bx - sn by + cx
    double cs_y, sn_y, cy_y;        // pose giving the y coordinates: sn bx + cs by + cy
    int active;
};

__device__ __forceinline__ void geo_pose(const GeoJob& J, int t) {
    if (t >= J.L.poly.m) return;
    double bx = J.body[2 * t], by = J.body[2 * t + 1];
    double* v = const_cast<double*>(J.L.poly.v);
    v[2 * t] = (J.cs_x * bx - J.sn_x * by) + J.cx_x;
    v[2 * t + 1] = (J.sn_y * bx + J.cs_y * by) + J.cy_y;
}

__device__ __forceinline__ int geo_nverts(const Box& r) { return (r.w() + 1) * (r.h() + 1); }
__device__ __forceinline__ int geo_nfaces(const Box& r) { return (r.w() + 1) * r.h() + r.w() * (r.h() + 1); }

// Phase 1 of the vertex classes: thread t of the job; true = left to phase 2.
// P: the job's polygon (its posed vertices, possibly in LDS).
__device__ __forceinline__ bool geo_vertices1(const Grid& g, const GeoJob& J, const Poly& P, int t) {
    int vw = J.reg.w() + 1;
    if (t >= geo_nverts(J.reg)) return false;
    int i = J.reg.i0 + t % vw, j = J.reg.j0 + t / vw;
    double px = vx_of(g, i), py = vy_of(g, j);
    int c = classify_quick(P, px, py);
    if (c < 0 && P.m <= SMALL_POLY) c = poly_classify<1>(P, px, py, 0);
    if (c < 0) return true;
    J.L.vcls[(size_t)j * (g.nx + 1) + i] = (int8_t)c;
    return false;
}
// Phase 2 of item t (one wavefront walks the polygon; the lanes share its edges).
__device__ __forceinline__ void geo_vertex_walk(const Grid& g, const GeoJob& J, const Poly& P, int t, int lane) {
    int vw = J.reg.w() + 1;
    int i = J.reg.i0 + t % vw, j = J.reg.j0 + t / vw;
    int c = poly_classify<WAVE>(P, vx_of(g, i), vy_of(g, j), lane);
    if (lane == 0) J.L.vcls[(size_t)j * (g.nx + 1) + i] = (int8_t)c;
}

// Vertex classes of a many-sided polygon, VT x VT vertices of the region per wavefront.
// Over the rectangle R spanned by a tile's vertices an edge's orientation value is affine
// in the vertex, so its exact least and greatest values are taken at corners of R; its
// rounding error is below 5 units in the last place of |dx| |py - ay| + |dy| |px - ax|,
// which is greatest at a corner as well.  An edge whose corner values clear twice that
// bound (with room to spare) is settled for the whole tile: negative at every vertex of R
// (every vertex of the tile is fluid), or non-negative at all of them (it cannot make any
// vertex fluid).  The tile's open vertices are then tested against the other edges only,
// with the formula of the full test, so every class equals that of the full test.
constexpr int VT = 8;
constexpr int UNC_CAP = 512;  // edges a tile tests vertex by vertex; beyond: the full test
__device__ void geo_vertex_tile(const Grid& g, const GeoJob& J, const Poly& P, int q, unsigned short* list,
                                int lane) {
    int vw = J.reg.w() + 1, vh = J.reg.h() + 1;
    int ntx = (vw + VT - 1) / VT;
    int ti = J.reg.i0 + (q % ntx) * VT, tj = J.reg.j0 + (q / ntx) * VT;
    int ie = min(ti + VT, J.reg.i0 + vw) - 1, je = min(tj + VT, J.reg.j0 + vh) - 1;  // last vertex of the tile
    int i = ti + lane % VT, j = tj + lane / VT;
    bool act = i <= ie && j <= je;
    double px = vx_of(g, i), py = vy_of(g, j);
    int c = act ? classify_quick(P, px, py) : FLUID;
    bool need = act && c < 0;
    if (__any(need)) {
        double x0 = vx_of(g, ti), x1 = vx_of(g, ie), y0 = vy_of(g, tj), y1 = vy_of(g, je);
        const double* v = P.v;
        int cnt = 0;
        bool neg = false;
        for (int base = 0; base < P.m; base += WAVE) {
            int k = base + lane;
            int cls = 0;  // 0: non-negative on R, 1: undecided, 2: negative on R
            if (k < P.m) {
                int k1 = k + 1 == P.m ? 0 : k + 1;
                double ax = v[2 * k], ay = v[2 * k + 1], bx = v[2 * k1], by = v[2 * k1 + 1];
                double o00 = orient(ax, ay, bx, by, x0, y0), o10 = orient(ax, ay, bx, by, x1, y0);
                double o01 = orient(ax, ay, bx, by, x0, y1), o11 = orient(ax, ay, bx, by, x1, y1);
                double my = fmax(fabs(y0 - ay), fabs(y1 - ay)), mx = fmax(fabs(x0 - ax), fabs(x1 - ax));
                double thr = (fabs(bx - ax) * my + fabs(by - ay) * mx) * 0x1p-48;
                double lo = fmin(fmin(o00, o10), fmin(o01, o11)), hi = fmax(fmax(o00, o10), fmax(o01, o11));
                cls = lo > thr ? 0 : (hi < -thr ? 2 : 1);
            }
            neg = neg || __any(cls == 2);
            unsigned long long mk = __ballot(cls == 1);
            int pos = cnt + __popcll(mk & ((1ull << lane) - 1ull));
            if (cls == 1 && pos < UNC_CAP) list[pos] = (unsigned short)k;
            cnt += __popcll(mk);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (need) {
            if (neg) {
                c = FLUID;
            } else if (cnt <= UNC_CAP) {
                // eight edges a round (their loads in flight together), the rest one by one
                bool out = false;
                int r = 0;
                for (; r + 8 <= cnt && !out; r += 8) {
                    uint4 w4 = *reinterpret_cast<const uint4*>(list + r);
                    unsigned int wd[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
                    for (int e = 0; e < 8; e++) {
                        int k = (int)((wd[e >> 1] >> (16 * (e & 1))) & 0xffffu);
                        int k1 = k + 1 == P.m ? 0 : k + 1;
                        out |= orient(v[2 * k], v[2 * k + 1], v[2 * k1], v[2 * k1 + 1], px, py) < 0.0;
                    }
                }
                for (; r < cnt && !out; r++) {
                    int k = list[r];
                    int k1 = k + 1 == P.m ? 0 : k + 1;
                    out = orient(v[2 * k], v[2 * k + 1], v[2 * k1], v[2 * k1 + 1], px, py) < 0.0;
                }
                c = out ? FLUID : SOLID;
            } else {
                c = poly_classify<1>(P, px, py, 0);
            }
        }
        __builtin_amdgcn_wave_barrier();  // the list is rewritten by the wavefront's next tile
    }
    if (act) J.L.vcls[(size_t)j * (g.nx + 1) + i] = (int8_t)c;
}
__device__ __forceinline__ int geo_vertex_tiles(const Box& r) {
    return ((r.w() + 1 + VT - 1) / VT) * ((r.h() + 1 + VT - 1) / VT);
}

// Face t of the region closure: x-faces first, then y-faces.
__device__ __forceinline__ void geo_face_ends(const Grid& g, const GeoJob& J, int t, bool& xf, int& i, int& j,
                                              double& ax, double& ay, int& ca, double& bx, double& by, int& cb) {
    int vw = J.reg.w() + 1, vh = J.reg.h() + 1;
    int nfx = vw * (vh - 1);
    const int8_t* vc = J.L.vcls;
    int W1 = g.nx + 1;
    xf = t < nfx;
    if (xf) {
        i = J.reg.i0 + t % vw;
        j = J.reg.j0 + t / vw;
        ax = bx = vx_of(g, i);
        ay = vy_of(g, j);
        by = vy_of(g, j + 1);
        ca = vc[(size_t)j * W1 + i];
        cb = vc[(size_t)(j + 1) * W1 + i];
    } else {
        t -= nfx;
        i = J.reg.i0 + t % (vw - 1);
        j = J.reg.j0 + t / (vw - 1);
        ax = vx_of(g, i);
        bx = vx_of(g, i + 1);
        ay = by = vy_of(g, j);
        ca = vc[(size_t)j * W1 + i];
        cb = vc[(size_t)j * W1 + i + 1];
    }
}
__device__ __forceinline__ void geo_store_face(const Grid& g, const GeoJob& J, bool xf, int i, int j, double2 iv) {
    if (xf) J.L.fx[(size_t)j * (g.nx + 1) + i] = iv;
    else J.L.fy[(size_t)j * g.nx + i] = iv;
}
// Face interval of item t: true = left to the chain search of a many-sided polygon.
__device__ __forceinline__ bool geo_faces1(const Grid& g, const GeoJob& J, int t) {
    if (t >= geo_nfaces(J.reg)) return false;
    bool xf;
    int i, j, ca, cb;
    double ax, ay, bx, by;
    geo_face_ends(g, J, t, xf, i, j, ax, ay, ca, bx, by, cb);
    double2 iv;
    if (!face_quick(J.L.poly, ax, ay, ca, bx, by, cb, iv)) {
        if (J.L.poly.m > SMALL_POLY) return true;
        iv = poly_seg_clip<1>(J.L.poly, ax, ay, bx, by, 0);
    }
    geo_store_face(g, J, xf, i, j, iv);
    return false;
}
// The same face by one wavefront's chain search on P (the polygon, possibly staged in LDS;
// every lane calls it).
__device__ __forceinline__ void geo_face_chain(const Grid& g, const GeoJob& J, const Poly& P, int t, int lane) {
    bool xf;
    int i, j, ca, cb;
    double ax, ay, bx, by;
    geo_face_ends(g, J, t, xf, i, j, ax, ay, ca, bx, by, cb);
    double2 iv = poly_seg_clip_chains(P, ax, ay, bx, by, lane);
    if (lane == 0) geo_store_face(g, J, xf, i, j, iv);
}

// The same face by its own thread (a polygon with monotone chains).
__device__ __forceinline__ void geo_face_thread(const Grid& g, const GeoJob& J, const Poly& P, int t) {
    bool xf;
    int i, j, ca, cb;
    double ax, ay, bx, by;
    geo_face_ends(g, J, t, xf, i, j, ax, ay, ca, bx, by, cb);
    geo_store_face(g, J, xf, i, j, poly_seg_clip_chains_t(P, ax, ay, bx, by));
}

// Volume fractions: open when all four faces are open, closed when all four are closed,
// otherwise 1 - (polygon area in the cell)/(hx hy); cut cells below the small-cell
// threshold count as solid.  true = left to the chain search of a many-sided polygon.
__device__ __forceinline__ double alpha_of_area(const Grid& g, double s) {
    double a = 1.0 - s / (g.hx * g.hy);
    if (a < 0.0) a = 0.0;
    if (a > 1.0) a = 1.0;
    if (a < g.alpha_min) a = 0.0;
    return a;
}
__device__ __forceinline__ bool geo_cells1(const Grid& g, const GeoJob& J, int t) {
    int cw = J.reg.w();
    if (t >= cw * J.reg.h()) return false;
    int i = J.reg.i0 + t % cw, j = J.reg.j0 + t / cw;
    const Level& L = J.L;
    double b[4] = {beta_x(g, L, i, j), beta_x(g, L, i + 1, j), beta_y(g, L, i, j), beta_y(g, L, i, j + 1)};
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
    } else if (L.poly.m > SMALL_POLY) {
        return true;
    } else {
        a = alpha_of_area(g, poly_clip_area<1>(L.poly, vx_of(g, i), vy_of(g, j), g.hx, g.hy, 0));
    }
    L.alpha[(size_t)j * g.nx + i] = a;
    return false;
}
// The same cell by one wavefront's chain search on P (every lane calls it).
__device__ __forceinline__ void geo_cell_chain(const Grid& g, const GeoJob& J, const Poly& P, int t, int lane) {
    int cw = J.reg.w();
    int i = J.reg.i0 + t % cw, j = J.reg.j0 + t / cw;
    double s = poly_clip_area_chains(P, vx_of(g, i), vy_of(g, j), g.hx, g.hy, lane);
    if (lane == 0) J.L.alpha[(size_t)j * g.nx + i] = alpha_of_area(g, s);
}

// The same cell by its own thread (a polygon with monotone chains).
__device__ __forceinline__ void geo_cell_thread(const Grid& g, const GeoJob& J, const Poly& P, int t) {
    int cw = J.reg.w();
    int i = J.reg.i0 + t % cw, j = J.reg.j0 + t / cw;
    J.L.alpha[(size_t)j * g.nx + i] = alpha_of_area(g, poly_clip_area_chains_t(P, vx_of(g, i), vy_of(g, j), g.hx, g.hy));
}

}  // namespace cc
