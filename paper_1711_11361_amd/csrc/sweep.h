// One directional sweep of the moving-boundary cut-cell method (Sec. 2.3.3-2.3.5):
// time-averaged apertures, states of cells that become fluid, wall Riemann problem and
// boundary flux, standard fluxes, stabilised shielded fluxes, conservative update and the
// covering of cells that become solid.
//
// Split of the work:
//   * the dense kernels update every cell outside the sweep box (the bodies' region grown
//     by three cells): there all stencil cells are regular, so the plain MUSCL-Hancock/HLLC
//     update applies; they stream the state once (read U_in, write U_out);
//   * the box phases (swept apertures, stage and wall, patch, cover, collapse rounds)
//     handle every cell of the sweep box with the general cut-cell formulas, through
//     box-local staging arrays.
// The phases are written as per-thread bodies; the launch wrappers map blocks of one
// launch onto the instances of a batch.
#pragma once
#include "cc_device.h"
#include "geometry.h"

namespace cc {
// Rigid map of the step restricted to one sweep direction and the body motion data.
struct Motion {
    double cosd, sind, c0x, c0y, c1x, c1y;  // M(X) = R (X - c0) + c1
    double vx, vy, thd, chx, chy;            // rigid velocity at mid-step: v + thd z x (X - ch)
};

// Box-local staging arrays of one sweep (capacity `cap` cells, `capf` faces).
struct Stage {
    double* Q;     // 4*cap: states used for fluxes
    double* U1;    // 4*cap: content after donations
    int8_t* has;   // cap
    double* bt;    // capf: time-averaged apertures of the faces normal to the sweep
    int8_t* wall;  // cap
    double* fb;    // 4*cap: boundary flux in the sweep direction
    double* wv;    // 4*cap: F^B - u_wall^d Q^B
    double* ahat;  // cap
    double* U2;    // 4*cap: updated content before covering
    int8_t* gone;  // cap: 1 covered, 2 collapsed
    int8_t* f1;    // cap: post-cover flags of the first collapse round (0 eligible, 1 bad, 2 out)
    int8_t* f2;    // cap: the same for the second round
    unsigned int* nbad;  // 2 counters: bad cells found before round 1 / round 2
    int cap;
};

struct Common {    // boundary state of the step's first sweep, per grid cell
    double* qb;    // 4*nc
    int32_t* stamp;
};

__device__ __forceinline__ int bidx(const Box& B, int i, int j) { return (j - B.j0) * B.w() + (i - B.i0); }

// Index of the d-face (i, j) in the box-local face array (x-faces: (w+1) per row; y-faces:
// w per row, h+1 rows).
template <int D>
__device__ __forceinline__ int fidx(const Box& B, int i, int j) {
    return D == 0 ? (j - B.j0) * (B.w() + 1) + (i - B.i0) : (j - B.j0) * B.w() + (i - B.i0);
}

__device__ __forceinline__ double step_disp(const Motion& M, int d, double x, double y) {
    double dx = x - M.c0x, dy = y - M.c0y;
    if (d == 0) return ((M.cosd * dx - M.sind * dy) + M.c1x) - x;
    return ((M.sind * dx + M.cosd * dy) + M.c1y) - y;
}

// One sweep of one instance.
struct SweepJob {
    Level Ls, Le;   // start and end levels
    Box B;          // sweep box (empty: no cut cells)
    const void* Uin;
    void* Uout;
    double lam;     // dt / h in the sweep direction
    int dir, first; // direction; 1 for the step's first sweep
};

// --------------------------------------------------------------- time-averaged apertures
// Exact average over the sweep of the aperture of a face normal to the sweep direction
// (Eq. timeAveragedBeta): the solid length integrated over the sweep is the area of the
// start polygon inside the strip swept across the face.
struct Strip {
    double x0, y0, sw, sh, w, hf;
};

// Settles face (i, j) without the polygon loop when possible (returns 1 with r set), else
// returns 0 with the strip to clip.
template <int D>
__device__ __forceinline__ int swept_quick(const Grid& g, const SweepJob& J, const Motion& M, int i, int j,
                                           double& r, Strip& st) {
    const Level& Ls = J.Ls;
    double bs = D == 0 ? beta_x(g, Ls, i, j) : beta_y(g, Ls, i, j);
    double be = D == 0 ? beta_x(g, J.Le, i, j) : beta_y(g, J.Le, i, j);
    if (bs == 0.0 && be == 0.0) {
        r = 0.0;
        return 1;
    }
    const Poly& P = Ls.poly;
    if (P.m == 0) {
        r = 0.5 * (bs + be);
        return 1;
    }
    double X = vx_of(g, i), Y = vy_of(g, j);
    double h = D == 0 ? g.hx : g.hy, hf = D == 0 ? g.hy : g.hx;
    double Dd = D == 0 ? step_disp(M, 0, X, Y + 0.5 * g.hy) : step_disp(M, 1, X + 0.5 * g.hx, Y);
    if (!(fabs(Dd) > 1e-12 * h)) {
        r = 0.5 * (bs + be);
        return 1;
    }
    double w = fabs(Dd);
    if (D == 0) {
        st.x0 = Dd > 0.0 ? X - Dd : X;
        st.y0 = Y;
        st.sw = w;
        st.sh = hf;
    } else {
        st.x0 = X;
        st.y0 = Dd > 0.0 ? Y - Dd : Y;
        st.sw = hf;
        st.sh = w;
    }
    st.w = w;
    st.hf = hf;
    if (st.x0 + st.sw < P.xmin || st.x0 > P.xmax || st.y0 + st.sh < P.ymin || st.y0 > P.ymax ||
        rect_outside_disc(P, st.x0, st.y0, st.sw, st.sh)) {
        r = 1.0;
        return 1;
    }
    return 0;
}

__device__ __forceinline__ double strip_beta(double a, const Strip& st) {
    double r = 1.0 - a / (st.w * st.hf);
    if (r < 0.0) r = 0.0;
    if (r > 1.0) r = 1.0;
    return r;
}

// Thread t over the box's faces normal to the sweep direction; true = left to the chain
// search of a many-sided polygon.
template <int D>
__device__ bool swept1(const Grid& g, const SweepJob& J, const Motion& M, const Stage& S, int t) {
    const Box& B = J.B;
    int fw = D == 0 ? B.w() + 1 : B.w(), fh = D == 0 ? B.h() : B.h() + 1;
    if (t >= fw * fh) return false;
    int i = B.i0 + t % fw, j = B.j0 + t / fw;
    double r;
    Strip st;
    if (!swept_quick<D>(g, J, M, i, j, r, st)) {
        if (J.Ls.poly.m > SMALL_POLY) return true;
        r = strip_beta(poly_clip_area<1>(J.Ls.poly, st.x0, st.y0, st.sw, st.sh, 0), st);
    }
    S.bt[fidx<D>(B, i, j)] = r;
    return false;
}

// The same face of a many-sided start polygon P (possibly staged in LDS) by one
// wavefront's chain search (every lane calls it).
template <int D>
__device__ void swept_chain(const Grid& g, const SweepJob& J, const Poly& P, const Motion& M, const Stage& S, int t,
                            int lane) {
    const Box& B = J.B;
    int fw = D == 0 ? B.w() + 1 : B.w();
    int i = B.i0 + t % fw, j = B.j0 + t / fw;
    double r;
    Strip st;
    swept_quick<D>(g, J, M, i, j, r, st);
    double a = poly_clip_area_chains(P, st.x0, st.y0, st.sw, st.sh, lane);
    if (lane == 0) S.bt[fidx<D>(B, i, j)] = strip_beta(a, st);
}

// The same face by its own thread (a start polygon with monotone chains).
template <int D>
__device__ void swept_thread(const Grid& g, const SweepJob& J, const Poly& P, const Motion& M, const Stage& S,
                             int t) {
    const Box& B = J.B;
    int fw = D == 0 ? B.w() + 1 : B.w();
    int i = B.i0 + t % fw, j = B.j0 + t / fw;
    double r;
    Strip st;
    swept_quick<D>(g, J, M, i, j, r, st);
    S.bt[fidx<D>(B, i, j)] = strip_beta(poly_clip_area_chains_t(P, st.x0, st.y0, st.sw, st.sh), st);
}

// ------------------------------------------------------------------ stage (donations)
// Oracle-order neighbour offsets: four face neighbours, then the diagonals.
__constant__ int c_d8[8][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}, {-1, -1}, {1, -1}, {-1, 1}, {1, 1}};

template <typename R>
__device__ __forceinline__ double ld_rho(const R* U, size_t nc, size_t k) { return (double)U[k]; }

// Donor set of receiver (i, j): face neighbours with alpha_s > 0 and content, else all
// eight neighbours.  Returns the count, fills the linear indices.
template <typename R>
__device__ int donors(const Grid& g, const Level& Ls, const R* U, int i, int j, int* don) {
    int nd = 0;
    for (int pass = 0; pass < 2 && nd == 0; pass++) {
        int cnt = pass == 0 ? 4 : 8;
        for (int q = 0; q < cnt; q++) {
            int ii = i + c_d8[q][0], jj = j + c_d8[q][1];
            if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny) continue;
            size_t kk = (size_t)jj * g.nx + ii;
            double a = Ls.alpha[kk], r = (double)U[kk];  // both loads in flight together
            if ((a > 0.0) & (r > 0.0)) don[nd++] = (int)kk;
        }
    }
    return nd;
}

// The donor set of receiver (i, j) as donors() finds it, with the sums of the donors'
// fractions and contents in donor order.  With FP32 state the face neighbours' fractions
// and contents are loaded in one round (the usual case); the eight-neighbour set, needed
// only when no face neighbour qualifies, goes through donors(), and so does every FP64
// state (its twenty loads in flight spill registers in the kernels this runs in).
template <typename R>
__device__ __forceinline__ int donor_sums(const Grid& g, const Level& Ls, const R* U, int i, int j, size_t nc,
                                          double& sa, double su[4]) {
    sa = 0.0;
    su[0] = su[1] = su[2] = su[3] = 0.0;
    if constexpr (sizeof(R) == 4) {
        double a[4], c[4][4];
        bool in[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            int ii = i + c_d8[q][0], jj = j + c_d8[q][1];
            in[q] = ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny;
            size_t kk = in[q] ? (size_t)jj * g.nx + ii : (size_t)j * g.nx + i;
            a[q] = Ls.alpha[kk];
#pragma unroll
            for (int m = 0; m < 4; m++) c[q][m] = (double)U[m * nc + kk];
        }
        int nd = 0;
#pragma unroll
        for (int q = 0; q < 4; q++)
            if (in[q] && (a[q] > 0.0) && (c[q][0] > 0.0)) {
                nd++;
                sa += a[q];
#pragma unroll
                for (int m = 0; m < 4; m++) su[m] += c[q][m];
            }
        if (nd > 0) return nd;
    }
    int don[8];
    int nd = donors(g, Ls, U, i, j, don);
    for (int qd = 0; qd < nd; qd++) sa += Ls.alpha[don[qd]];
    for (int m = 0; m < 4; m++)
        for (int qd = 0; qd < nd; qd++) su[m] += (double)U[m * nc + don[qd]];
    return nd;
}

// ------------------------------------------------------------------ wall quantities
// The solid intervals of the four faces of cell (i, j) in a level: x-faces i and i + 1,
// y-faces j and j + 1 (loaded together, so that their latencies overlap).
struct CellFaces {
    double2 f[4];
};
__device__ __forceinline__ CellFaces cell_faces(const Grid& g, const Level& L, int i, int j) {
    CellFaces c;
    c.f[0] = L.fx[(size_t)j * (g.nx + 1) + i];
    c.f[1] = L.fx[(size_t)j * (g.nx + 1) + i + 1];
    c.f[2] = L.fy[(size_t)j * g.nx + i];
    c.f[3] = L.fy[(size_t)(j + 1) * g.nx + i];
    return c;
}
__device__ __forceinline__ bool cell_cut_f(const CellFaces& c) {
    int ones = 0, zeros = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        double b = interval_beta(c.f[k]);
        ones += b == 1.0;
        zeros += b == 0.0;
    }
    return ones != 4 && zeros != 4;
}

// Mean of the boundary crossing points on the cell's faces; cell centre if none.
__device__ void wall_point(const Grid& g, const CellFaces& c, int i, int j, double* wx, double* wy) {
    double sx = 0.0, sy = 0.0;
    int n = 0;
#pragma unroll
    for (int e = 0; e < 4; e++) {
        double2 iv = c.f[e];
        double ox, oy, dx, dy;
        if (e < 2) {
            ox = vx_of(g, i + e);
            oy = vy_of(g, j);
            dx = 0.0;
            dy = g.hy;
        } else {
            ox = vx_of(g, i);
            oy = vy_of(g, j + e - 2);
            dx = g.hx;
            dy = 0.0;
        }
        if (!(iv.y > iv.x)) continue;
        double tt[2] = {iv.x, iv.y};
        for (int q = 0; q < 2; q++) {
            double tq = tt[q];
            if (tq > 0.0 && tq < 1.0) {
                sx += ox + tq * dx;
                sy += oy + tq * dy;
                n++;
            }
        }
    }
    if (n == 0) {
        *wx = vx_of(g, i) + 0.5 * g.hx;
        *wy = vy_of(g, j) + 0.5 * g.hy;
        return;
    }
    *wx = sx / (double)n;
    *wy = sy / (double)n;
}

// Wall Riemann problem along the unit normal (into the solid): the cell state against its
// mirror image moving with the wall (Eq. riemann_wallvel), HLLC/Davis star pressure and
// density; the star pressure is not allowed below zero.
__device__ __forceinline__ void wall_riemann(const double q[4], double nx, double ny, double wx, double wy,
                                             double g, double* pst, double* rst) {
    double r = q[0];
    double u = q[1] / r, v = q[2] / r;
    double p = pressure(q, g);
    double a = sqrt(g * p / r);
    double un = u * nx + v * ny;
    double wn = wx * nx + wy * ny;
    double ul = un, ur = 2.0 * wn - un;
    double sl = fmin(ul - a, ur - a);
    double sr = fmax(ul + a, ur + a);
    double ss = (p - p + r * ul * (sl - ul) - r * ur * (sr - ur)) / (r * (sl - ul) - r * (sr - ur));
    double ps = p + r * (sl - ul) * (ss - ul);
    double rs = r * (sl - ul) / (sl - ss);
    if (ps < 0.0) ps = 0.0;
    *pst = ps;
    *rst = rs;
}

// States of the box cells before the sweep (Eqs. volumeWeighting, cutCellInitialisation,
// cutCellInitialisationDonorCellUpdate as read for exact time averages):
//   uncovered (alpha_s = 0 < alpha_e): state = donors' volume-weighted average, no content;
//   emptied (alpha_s > 0, no content): content sigma * sum(donor content);
//   donors of emptied cells keep the fraction (1 - sum sigma) of their content.
// Then the cell's wall quantities: wall flag, shielded volume, boundary flux F^B (advective
// part from the step's common boundary state, pressure part from this stage) and
// F^B - u_wall^d Q^B.
// Body of wall cell k in a sweep of a context with several bodies: the one cutting it at
// level s (when cut there), else at level e; status bit 4 when the two levels' differ.
__device__ __forceinline__ int wall_body(const SweepJob& J, size_t k, bool cs, bool ce, unsigned int* status) {
    int bs = J.Ls.cbody[k], be = J.Le.cbody[k];
    if (cs && ce && bs >= 0 && be >= 0 && bs != be) atomicOr(status, 4u);
    return cs && bs >= 0 ? bs : (be >= 0 ? be : 0);
}

// MB: several bodies, the wall velocity from the motion bm[] of the cell's body (else M).
template <int D, typename R, bool MB = false>
__device__ void stagewall(const Grid& g, const SweepJob& J, const Motion& M, const Stage& S, const Common& C,
                          unsigned int* status, int32_t step_id, int t, const Motion* bm = nullptr) {
    const Level& Ls = J.Ls;
    const Level& Le = J.Le;
    const Box& B = J.B;
    const R* U = (const R*)J.Uin;
    int first = J.first;
    if (t >= B.w() * B.h()) return;
    int i = B.i0 + t % B.w(), j = B.j0 + t / B.w();
    size_t nc = (size_t)g.nx * g.ny, k = (size_t)j * g.nx + i;
    int cap = S.cap;
    // everything the cell's own quantities need, loaded up front
    double as = Ls.alpha[k], ae = Le.alpha[k];
    double u[4];
#pragma unroll
    for (int m = 0; m < 4; m++) u[m] = (double)U[m * nc + k];
    CellFaces fs = cell_faces(g, Ls, i, j), fe = cell_faces(g, Le, i, j);
    double bt_lo = S.bt[fidx<D>(B, i, j)];
    double bt_hi = D == 0 ? S.bt[fidx<0>(B, i + 1, j)] : S.bt[fidx<1>(B, i, j + 1)];
    int32_t stamp = C.stamp[k];
    double qb_old[4];
#pragma unroll
    for (int m = 0; m < 4; m++) qb_old[m] = C.qb[m * nc + k];
    bool uncovered = as == 0.0 && ae > 0.0;
    bool emptied = as > 0.0 && ae > 0.0 && !(u[0] > 0.0);
    double q[4] = {0, 0, 0, 0};
    double u1[4] = {u[0], u[1], u[2], u[3]};
    int has = 0;
    if (uncovered || emptied) {
        double sa, su[4];
        int nd = donor_sums(g, Ls, U, i, j, nc, sa, su);
        if (nd == 0) {
            atomicOr(status, 1u);
        } else if (uncovered) {
            for (int m = 0; m < 4; m++) q[m] = su[m] / sa;
            has = 1;
            u1[0] = u1[1] = u1[2] = u1[3] = 0.0;
        } else {
            double sig = as / (as + sa);
            for (int m = 0; m < 4; m++) u1[m] = sig * su[m];
        }
    } else if (as > 0.0 && u[0] > 0.0) {
        // a live cell may donate to emptied neighbours (visited in increasing cell order);
        // the neighbours' fractions and densities are loaded together first, all three
        // unconditionally (a short-circuit test would make each load wait for the one
        // before; indices clamped into the grid, the ones outside it are skipped below)
        unsigned emptied = 0u;  // bit q: neighbour q (row-major in the 3 x 3 block) is emptied
#pragma unroll
        for (int q = 0; q < 9; q++) {
            int li = min(max(i + q % 3 - 1, 0), g.nx - 1), lj = min(max(j + q / 3 - 1, 0), g.ny - 1);
            size_t l = (size_t)lj * g.nx + li;
            double a_s = Ls.alpha[l], a_e = Le.alpha[l], r = (double)U[l];
            if ((a_s > 0.0) & (a_e > 0.0) & !(r > 0.0)) emptied |= 1u << q;
        }
        double take = 0.0;
        for (int dj = -1; dj <= 1; dj++)
            for (int di = -1; di <= 1; di++) {
                if (di == 0 && dj == 0) continue;
                int li = i + di, lj = j + dj;
                if (li < 0 || li >= g.nx || lj < 0 || lj >= g.ny) continue;
                if (!((emptied >> ((dj + 1) * 3 + (di + 1))) & 1u)) continue;
                double asl = Ls.alpha[(size_t)lj * g.nx + li];
                int don[8];
                int nd = donors(g, Ls, U, li, lj, don);
                bool mine = false;
                double sa = 0.0;
                for (int qd = 0; qd < nd; qd++) {
                    sa += Ls.alpha[don[qd]];
                    mine |= don[qd] == (int)k;
                }
                if (mine) take += asl / (asl + sa);
            }
        if (take > 0.0)
            for (int m = 0; m < 4; m++) u1[m] = u[m] * (1.0 - take);
    }
    if (!has && as > 0.0 && u1[0] > 0.0) {
        has = 1;
        for (int m = 0; m < 4; m++) q[m] = u1[m] / as;
    }
    int b = bidx(B, i, j);
    for (int m = 0; m < 4; m++) {
        S.Q[m * cap + b] = q[m];
        S.U1[m * cap + b] = u1[m];
    }
    S.has[b] = (int8_t)has;
    double ab = 0.5 * (as + ae);
    double bw, be, bs, bn;
    if (D == 0) {
        bw = bt_lo;
        be = bt_hi;
        bs = 0.5 * (interval_beta(fs.f[2]) + interval_beta(fe.f[2]));
        bn = 0.5 * (interval_beta(fs.f[3]) + interval_beta(fe.f[3]));
    } else {
        bw = 0.5 * (interval_beta(fs.f[0]) + interval_beta(fe.f[0]));
        be = 0.5 * (interval_beta(fs.f[1]) + interval_beta(fe.f[1]));
        bs = bt_lo;
        bn = bt_hi;
    }
    double Nx = (bw - be) * g.hy, Ny = (bs - bn) * g.hx;
    bool wall = ab > 0.0 && (Nx != 0.0 || Ny != 0.0);
    double fb[4] = {0, 0, 0, 0}, wv[4] = {0, 0, 0, 0}, ahat = 0.0;
    if (wall) {
        // unit normal: the time average of the wall's unit normal over the sweep (end of
        // Sec. 2.3.4), the normalised sum of the start and end levels' unit normals, each
        // from that level's apertures (exact for a planar wall); a level where the cell has
        // no wall adds nothing; without either, the effective vector's direction
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int lv = 0; lv < 2; lv++) {
            const CellFaces& f = lv == 0 ? fs : fe;
            double lx = (interval_beta(f.f[0]) - interval_beta(f.f[1])) * g.hy;
            double ly = (interval_beta(f.f[2]) - interval_beta(f.f[3])) * g.hx;
            double ll = sqrt(lx * lx + ly * ly);
            if (ll > 0.0) {
                sx += lx / ll;
                sy += ly / ll;
            }
        }
        double nn = sqrt(sx * sx + sy * sy);
        if (!(nn > 0.0)) {
            sx = Nx;
            sy = Ny;
            nn = sqrt(Nx * Nx + Ny * Ny);
        }
        double nxu = sx / nn, nyu = sy / nn;
        double wx, wy;
        bool cs = cell_cut_f(fs), ce = cell_cut_f(fe);
        if (cs && ce) {
            double ax, ay, bx2, by2;
            wall_point(g, fs, i, j, &ax, &ay);
            wall_point(g, fe, i, j, &bx2, &by2);
            wx = 0.5 * (ax + bx2);
            wy = 0.5 * (ay + by2);
        } else if (cs) {
            wall_point(g, fs, i, j, &wx, &wy);
        } else {
            wall_point(g, fe, i, j, &wx, &wy);
        }
        const Motion& Mw = MB ? bm[wall_body(J, k, cs, ce, status)] : M;
        double uwx = Mw.vx - Mw.thd * (wy - Mw.chy);
        double uwy = Mw.vy + Mw.thd * (wx - Mw.chx);
        double blo = D == 0 ? bw : bs, bhi = D == 0 ? be : bn;
        double mn = blo < bhi ? blo : bhi;
        double sh = fabs(bhi - blo);
        double ah = ab - mn;
        if (ah < 0.0) ah = 0.0;
        if (ah > sh) ah = sh;
        ahat = ah;
        if (has) {
            double pst, rst;
            wall_riemann(q, nxu, nyu, uwx, uwy, g.gamma, &pst, &rst);
            double u = q[1] / q[0], v = q[2] / q[0];
            double un = u * nxu + v * nyu, wn = uwx * nxu + uwy * nyu;
            double usx = (u - un * nxu) + wn * nxu;
            double usy = (v - un * nyu) + wn * nyu;
            double qb[4];
            if (first || stamp != step_id) {
                qb[0] = rst;
                qb[1] = rst * usx;
                qb[2] = rst * usy;
                qb[3] = pst / (g.gamma - 1.0) + 0.5 * rst * (usx * usx + usy * usy);
                if (first) {
                    for (int m = 0; m < 4; m++) C.qb[m * nc + k] = qb[m];
                    C.stamp[k] = step_id;
                }
            } else {
                for (int m = 0; m < 4; m++) qb[m] = qb_old[m];
            }
            double ua = (D == 0 ? qb[1] : qb[2]) / qb[0];
            double us = D == 0 ? usx : usy;
            fb[0] = ua * qb[0];
            fb[1] = ua * qb[1] + (D == 0 ? pst : 0.0);
            fb[2] = ua * qb[2] + (D == 1 ? pst : 0.0);
            fb[3] = ua * qb[3] + pst * us;
            double ud = D == 0 ? uwx : uwy;
            for (int m = 0; m < 4; m++) wv[m] = fb[m] - ud * qb[m];
        }
    }
    S.wall[b] = (int8_t)wall;
    S.ahat[b] = ahat;
    for (int m = 0; m < 4; m++) {
        S.fb[m * cap + b] = fb[m];
        S.wv[m * cap + b] = wv[m];
    }
}

// ------------------------------------------------------------------ budget slots
// Conservation budget of a sweep (Sec. 3.3: the change of the totals is what crossed the
// domain boundary, plus the wall pressure terms, minus residuals that found no recipient).
// Blocks that own such terms write partial sums to slots of their own (no atomics); the
// member's collapse block adds the slots up in a fixed order at the end of the sweep.
// Layout of a member's slot array (doubles):
//   [0]                     number of dense boundary slots the sweep's dense launch wrote
//                           (two per line of the sweep)
//   [BS_DENSE + 4 k + m]    dense boundary slot k = 2 line + side: the flux of component m
//                           through the line's low (side 0) or high (side 1) domain face
//                           when the dense tiles update that cell, else 0
//   [bs_patch + 12 b + ...] patch segment b: low face, high face (as above), wall terms
//   [bs_cover + 4 b + m]    covering block b: residual without recipients
constexpr int BS_DENSE = 8;
struct BudgetSlots {
    double* base;  // null: the budget is not tracked
    int patch, cover;  // offsets of the patch and covering parts
};

// ------------------------------------------------------------------ patch (box update)
struct CellData {
    double q[4];
    double u1[4];
    bool has;
};

// State of the cell at line position p (ghost cells beyond the domain: zero-gradient copy
// or mirror with negated normal momentum).
template <int D, typename R>
__device__ __forceinline__ void fetch_cell(const Grid& g, const R* U, const Box& B, const Stage& S, int line, int p,
                                           int n, CellData& c) {
    int bc = p < 0 ? g.bc[D == 0 ? 0 : 2] : g.bc[D == 0 ? 1 : 3];
    int src = p;
    bool mirror = false;
    if (p < 0) {
        src = bc == 1 ? -1 - p : 0;
        mirror = bc == 1;
    } else if (p >= n) {
        src = bc == 1 ? 2 * n - 1 - p : n - 1;
        mirror = bc == 1;
    }
    if (src < 0) src = 0;
    if (src >= n) src = n - 1;
    int i = D == 0 ? src : line, j = D == 0 ? line : src;
    size_t nc = (size_t)g.nx * g.ny;
    // values are selected, not stored conditionally, so that the cell records stay in
    // registers
    bool in = B.has(i, j);
    int b = in ? bidx(B, i, j) : 0;
    size_t k = (size_t)j * g.nx + i;
    bool has = in ? S.has[b] != 0 : true;
    double q[4], u1[4];
    if (in) {
#pragma unroll
        for (int m = 0; m < 4; m++) {
            q[m] = S.Q[m * S.cap + b];
            u1[m] = S.U1[m * S.cap + b];
        }
    } else {
#pragma unroll
        for (int m = 0; m < 4; m++) q[m] = u1[m] = (double)U[m * nc + k];
    }
#pragma unroll
    for (int m = 0; m < 4; m++) q[m] = has ? q[m] : 0.0;
    if (mirror) q[1 + D] = -q[1 + D];
    c.has = has;
#pragma unroll
    for (int m = 0; m < 4; m++) {
        c.q[m] = q[m];
        c.u1[m] = u1[m];
    }
}

template <int D>
__device__ __forceinline__ double face_bt(const Box& B, const Stage& S, int line, int f) {
    int i = D == 0 ? f : line, j = D == 0 ? line : f;
    bool in = D == 0 ? (i >= B.i0 && i <= B.i1 && j >= B.j0 && j < B.j1)
                     : (i >= B.i0 && i < B.i1 && j >= B.j0 && j <= B.j1);
    return in ? S.bt[fidx<D>(B, i, j)] : 1.0;
}

struct WallData {
    bool wall;
    double ahat;
    double fb[4], wv[4];
};

template <int D>
__device__ __forceinline__ void fetch_wall(const Box& B, const Stage& S, int line, int p, int n, WallData& w) {
    w.wall = false;
    if (p < 0 || p >= n) return;
    int i = D == 0 ? p : line, j = D == 0 ? line : p;
    if (!B.has(i, j)) return;
    int b = bidx(B, i, j);
    w.wall = S.wall[b] != 0;
    w.ahat = S.ahat[b];
    for (int m = 0; m < 4; m++) {
        w.fb[m] = S.fb[m * S.cap + b];
        w.wv[m] = S.wv[m * S.cap + b];
    }
}

// Stabilised aperture-weighted flux of face f (Eqs. Klein2shieldedFluxMethod2,
// Klein2DtotalfluxaMethod2 in division-free form, shielded flux of the same face):
// Phi = bt F - kap (s_L - ahat_L)(F - FB_L) - kap (s_R - ahat_R)(F - FB_R).
template <int D>
__device__ __forceinline__ void face_phi(double bt, double btm, double btp, const double* er_l, const double* el_r, bool act,
                         const WallData& L, const WallData& Rw, bool l_in, bool r_in, double gam, double* phi) {
    if (!act) {
        for (int m = 0; m < 4; m++) phi[m] = 0.0;
        return;
    }
    double F[4];
    hllc<double, D>(er_l, el_r, gam, F);
    double sL = 0.0, sR = 0.0;
    if (l_in && L.wall) {
        double d = bt - btm;
        sL = d > 0.0 ? d : 0.0;
    }
    if (r_in && Rw.wall) {
        double d = bt - btp;
        sR = d > 0.0 ? d : 0.0;
    }
    double kap = 1.0;
    if (sL + sR > bt) kap = bt / (sL + sR);
    double cL = sL > 0.0 ? kap * (sL - L.ahat) : 0.0;
    double cR = sR > 0.0 ? kap * (sR - Rw.ahat) : 0.0;
    for (int m = 0; m < 4; m++) {
        double v = bt * F[m];
        if (cL != 0.0) v = v - cL * (F[m] - L.fb[m]);
        if (cR != 0.0) v = v - cR * (F[m] - Rw.fb[m]);
        phi[m] = v;
    }
}

// Update of every box cell (Eqs. Klein2DcompleteMovingMethod2a/b): content plus
// dt/h (Phi_lo - Phi_hi + W), W = (beta_hi - beta_lo)(F^B - u_wall^d Q^B) for wall cells;
// then covered cells and collapsed cells (inadmissible update) are marked for emptying.
template <int D, typename R>
__device__ void patch(const Grid& g, const SweepJob& J, const Stage& S, unsigned int* ncollapse, int t) {
    const Level& Ls = J.Ls;
    const Level& Le = J.Le;
    const Box& B = J.B;
    const R* U = (const R*)J.Uin;
    double lam = J.lam;
    if (t >= B.w() * B.h()) return;
    int i = B.i0 + t % B.w(), j = B.j0 + t / B.w();
    int n = D == 0 ? g.nx : g.ny;
    int line = D == 0 ? j : i, p = D == 0 ? i : j;
    int b = bidx(B, i, j), cap = S.cap;
    size_t k = (size_t)j * g.nx + i;
    double gam = g.gamma;
    double as = Ls.alpha[k], ae = Le.alpha[k];
    double u2[4] = {0, 0, 0, 0};
    bool has_c = S.has[b] != 0;
    if (has_c) {
        CellData c[5];
        // fully unrolled, so that the small arrays stay in registers
#pragma unroll
        for (int s = 0; s < 5; s++) fetch_cell<D>(g, U, B, S, line, p - 2 + s, n, c[s]);
        double el[3][4], er[3][4];
#pragma unroll
        for (int s = 1; s <= 3; s++) {
            bool ok = c[s - 1].has && c[s + 1].has;
            if (c[s].has) muscl<double, D>(c[s - 1].q, c[s].q, c[s + 1].q, ok, lam, gam, el[s - 1], er[s - 1]);
        }
        double bt[4];  // faces p-1, p, p+1, p+2
#pragma unroll
        for (int s = 0; s < 4; s++) bt[s] = face_bt<D>(B, S, line, p - 1 + s);
        WallData w[3];
#pragma unroll
        for (int s = 0; s < 3; s++) fetch_wall<D>(B, S, line, p - 1 + s, n, w[s]);
        double plo[4], phi_hi[4];
        bool act_lo = bt[1] > 0.0 && c[1].has && c[2].has;
        bool act_hi = bt[2] > 0.0 && c[2].has && c[3].has;
        face_phi<D>(bt[1], bt[0], bt[2], er[0], el[1], act_lo, w[0], w[1], p > 0, true, gam, plo);
        face_phi<D>(bt[2], bt[1], bt[3], er[1], el[2], act_hi, w[1], w[2], true, p + 1 < n, gam, phi_hi);
        double W[4] = {0, 0, 0, 0};
        if (w[1].wall) {
            double db = bt[2] - bt[1];
            for (int m = 0; m < 4; m++) W[m] = db * w[1].wv[m];
        }
        for (int m = 0; m < 4; m++) u2[m] = c[2].u1[m] + lam * ((plo[m] - phi_hi[m]) + W[m]);
    }
    int gone = 0;
    if (as > 0.0 && ae == 0.0) {
        gone = 1;
    } else if (ae > 0.0 && has_c) {
        double r = u2[0], e = u2[3];
        if (!(r > 0.0) || !(e - 0.5 * (u2[1] * u2[1] + u2[2] * u2[2]) / r > 0.0)) {
            gone = 2;
            atomicAdd(ncollapse, 1u);
        }
    }
    for (int m = 0; m < 4; m++) S.U2[m * cap + b] = u2[m];
    S.gone[b] = (int8_t)gone;
}


// The same update by line segments: a block of PL_T threads covers PL_OUT consecutive box
// cells of one line in the sweep direction plus two cells each side; every thread fetches
// one cell, and each cell's reconstruction and each face's stabilised flux are computed
// once and exchanged through LDS (the per-cell form above computes three reconstructions
// and two face fluxes per cell).  Face f lies between cells f-1 and f; its flux takes the
// left cell as inside the domain when f > 0 and the right one when f < n, which is what
// the per-cell form passes for a cell's lower and upper face.  Results are identical.
constexpr int PL_T = 64;
constexpr int PL_OUT = PL_T - 4;

template <int D>
__host__ __device__ constexpr int patch_line_blocks(int capw, int caph) {
    return D == 0 ? caph * ((capw + PL_OUT - 1) / PL_OUT) : capw * ((caph + PL_OUT - 1) / PL_OUT);
}

struct PatchLds {
    double q[4][PL_T];
    double er[4][PL_T];
    double phi[4][PL_T];
    bool has[PL_T];
};

// lb: the block's index within the member (uniform over the block; every thread calls it).
// bs: budget slots (base null: not tracked): the block's slot gets the stabilised fluxes
// through the domain's low and high faces of its line (when it updates the end cells) and
// the sum of its cells' wall terms.
template <int D, typename R>
__device__ void patch_line(const Grid& g, const SweepJob& J, const Stage& S, unsigned int* ncollapse, int lb,
                           PatchLds& sh, const BudgetSlots& bs) {
    const Level& Ls = J.Ls;
    const Level& Le = J.Le;
    const Box& B = J.B;
    const R* U = (const R*)J.Uin;
    double lam = J.lam;
    int len = D == 0 ? B.w() : B.h();
    int nlines = D == 0 ? B.h() : B.w();
    int segs = (len + PL_OUT - 1) / PL_OUT;
    if (lb >= nlines * segs) return;  // uniform over the block
    int line = (D == 0 ? B.j0 : B.i0) + lb / segs;
    int first = D == 0 ? B.i0 : B.j0;
    int x = threadIdx.x;
    int p = first + (lb % segs) * PL_OUT - 2 + x;  // this thread's cell along the line
    int n = D == 0 ? g.nx : g.ny;
    double gam = g.gamma;
    CellData c;
    fetch_cell<D>(g, U, B, S, line, p, n, c);
#pragma unroll
    for (int m = 0; m < 4; m++) sh.q[m][x] = c.q[m];
    sh.has[x] = c.has;
    __syncthreads();
    double el[4] = {0, 0, 0, 0}, er[4] = {0, 0, 0, 0};
    if (x >= 1 && x < PL_T - 1 && c.has) {
        double qm[4], qp[4];
#pragma unroll
        for (int m = 0; m < 4; m++) {
            qm[m] = sh.q[m][x - 1];
            qp[m] = sh.q[m][x + 1];
        }
        bool ok = sh.has[x - 1] && sh.has[x + 1];
        muscl<double, D>(qm, c.q, qp, ok, lam, gam, el, er);
    }
#pragma unroll
    for (int m = 0; m < 4; m++) sh.er[m][x] = er[m];
    __syncthreads();
    WallData wl, wr;
    fetch_wall<D>(B, S, line, p, n, wr);
    double btf = 1.0, btp = 1.0;
    if (x >= 2 && x < PL_T - 1) {  // faces 2 .. PL_T-2: the lower and upper faces of the updated cells
        double btm = face_bt<D>(B, S, line, p - 1);
        btf = face_bt<D>(B, S, line, p);
        btp = face_bt<D>(B, S, line, p + 1);
        fetch_wall<D>(B, S, line, p - 1, n, wl);
        double erl[4], phi[4];
#pragma unroll
        for (int m = 0; m < 4; m++) erl[m] = sh.er[m][x - 1];
        bool act = btf > 0.0 && sh.has[x - 1] && c.has;
        face_phi<D>(btf, btm, btp, erl, el, act, wl, wr, p > 0, p < n, gam, phi);
#pragma unroll
        for (int m = 0; m < 4; m++) sh.phi[m][x] = phi[m];
    }
    __syncthreads();
    bool mine = !(x < 2 || x >= PL_T - 2 || p >= first + len);  // a cell this block updates
    double W[4] = {0, 0, 0, 0};
    if (mine && c.has && wr.wall) {
        double db = btp - btf;
        for (int m = 0; m < 4; m++) W[m] = db * wr.wv[m];
    }
    if (bs.base) {  // one wavefront: lane sums in a fixed order
        double* slot = bs.base + bs.patch + 12 * lb;
#pragma unroll
        for (int m = 0; m < 4; m++) {
            double lo = wave_sum(mine && p == 0 ? sh.phi[m][x] : 0.0);
            double hi = wave_sum(mine && p == n - 1 ? sh.phi[m][x + 1] : 0.0);
            double wt = wave_sum(W[m]);
            if (x == 0) {
                slot[m] = lo;
                slot[4 + m] = hi;
                slot[8 + m] = wt;
            }
        }
    }
    if (!mine) return;
    int i = D == 0 ? p : line, j = D == 0 ? line : p;
    int b = bidx(B, i, j), cap = S.cap;
    size_t k = (size_t)j * g.nx + i;
    double as = Ls.alpha[k], ae = Le.alpha[k];
    double u2[4] = {0, 0, 0, 0};
    if (c.has)
        for (int m = 0; m < 4; m++) u2[m] = c.u1[m] + lam * ((sh.phi[m][x] - sh.phi[m][x + 1]) + W[m]);
    int gone = 0;
    if (as > 0.0 && ae == 0.0) {
        gone = 1;
    } else if (ae > 0.0 && c.has) {
        double r = u2[0], e = u2[3];
        if (!(r > 0.0) || !(e - 0.5 * (u2[1] * u2[1] + u2[2] * u2[2]) / r > 0.0)) {
            gone = 2;
            atomicAdd(ncollapse, 1u);
        }
    }
    for (int m = 0; m < 4; m++) S.U2[m * cap + b] = u2[m];
    S.gone[b] = (int8_t)gone;
}

// The y sweep's patch update by tiles: a block of PT_C x PT_P threads covers PT_C adjacent
// box columns over PT_OUT consecutive rows, plus two rows each side; thread (c, r) fetches
// the cell of column c at row r, so that a row of the tile is PT_C consecutive cells of the
// row-major arrays (the line segments of patch_line would walk a column with one cell per
// cache line).  The per-cell and per-face work, and its order, are patch_line's: results
// are identical.
constexpr int PT_C = 16, PT_P = 16, PT_OUT = PT_P - 4, PT_T = PT_C * PT_P;

__host__ __device__ constexpr int patch_tile_blocks(int capw, int caph) {
    return ((capw + PT_C - 1) / PT_C) * ((caph + PT_OUT - 1) / PT_OUT);
}

struct TileLds {
    double q[4][PT_P][PT_C];
    double er[4][PT_P][PT_C];
    double phi[4][PT_P][PT_C];
    bool has[PT_P][PT_C];
    double red[12][PT_T / 64];
};

// lb: the block's index within the member (uniform over the block; every thread calls it).
// bs: budget slots as for patch_line (the tile's sums, its wavefronts in order).
template <typename R>
__device__ void patch_tile_y(const Grid& g, const SweepJob& J, const Stage& S, unsigned int* ncollapse, int lb,
                             TileLds& sh, const BudgetSlots& bs) {
    constexpr int D = 1;
    const Level& Ls = J.Ls;
    const Level& Le = J.Le;
    const Box& B = J.B;
    const R* U = (const R*)J.Uin;
    double lam = J.lam;
    int len = B.h();
    int ncb = (B.w() + PT_C - 1) / PT_C, segs = (len + PT_OUT - 1) / PT_OUT;
    if (lb >= ncb * segs) return;  // uniform over the block
    int cx = (int)threadIdx.x % PT_C, x = (int)threadIdx.x / PT_C;  // column in the tile, position along it
    int col = B.i0 + (lb % ncb) * PT_C + cx;
    bool colok = col < B.i1;
    int line = colok ? col : B.i1 - 1;  // columns past the box fetch a box column and update nothing
    int first = B.j0;
    int p = first + (lb / ncb) * PT_OUT - 2 + x;  // this thread's cell along the column
    int n = g.ny;
    double gam = g.gamma;
    CellData c;
    fetch_cell<D>(g, U, B, S, line, p, n, c);
#pragma unroll
    for (int m = 0; m < 4; m++) sh.q[m][x][cx] = c.q[m];
    sh.has[x][cx] = c.has;
    __syncthreads();
    double el[4] = {0, 0, 0, 0}, er[4] = {0, 0, 0, 0};
    if (x >= 1 && x < PT_P - 1 && c.has) {
        double qm[4], qp[4];
#pragma unroll
        for (int m = 0; m < 4; m++) {
            qm[m] = sh.q[m][x - 1][cx];
            qp[m] = sh.q[m][x + 1][cx];
        }
        bool ok = sh.has[x - 1][cx] && sh.has[x + 1][cx];
        muscl<double, D>(qm, c.q, qp, ok, lam, gam, el, er);
    }
#pragma unroll
    for (int m = 0; m < 4; m++) sh.er[m][x][cx] = er[m];
    __syncthreads();
    WallData wl, wr;
    fetch_wall<D>(B, S, line, p, n, wr);
    double btf = 1.0, btp = 1.0;
    if (x >= 2 && x < PT_P - 1) {  // the lower and upper faces of the updated cells
        double btm = face_bt<D>(B, S, line, p - 1);
        btf = face_bt<D>(B, S, line, p);
        btp = face_bt<D>(B, S, line, p + 1);
        fetch_wall<D>(B, S, line, p - 1, n, wl);
        double erl[4], phi[4];
#pragma unroll
        for (int m = 0; m < 4; m++) erl[m] = sh.er[m][x - 1][cx];
        bool act = btf > 0.0 && sh.has[x - 1][cx] && c.has;
        face_phi<D>(btf, btm, btp, erl, el, act, wl, wr, p > 0, p < n, gam, phi);
#pragma unroll
        for (int m = 0; m < 4; m++) sh.phi[m][x][cx] = phi[m];
    }
    __syncthreads();
    bool mine = colok && !(x < 2 || x >= PT_P - 2 || p >= first + len);  // a cell this block updates
    double W[4] = {0, 0, 0, 0};
    if (mine && c.has && wr.wall) {
        double db = btp - btf;
        for (int m = 0; m < 4; m++) W[m] = db * wr.wv[m];
    }
    if (bs.base) {  // per wavefront in a fixed lane order, then the wavefronts in order
        int wv = (int)threadIdx.x >> 6;
#pragma unroll
        for (int m = 0; m < 4; m++) {
            double lo = wave_sum(mine && p == 0 ? sh.phi[m][x][cx] : 0.0);
            double hi = wave_sum(mine && p == n - 1 ? sh.phi[m][x + 1][cx] : 0.0);
            double wt = wave_sum(W[m]);
            if ((threadIdx.x & 63) == 0) {
                sh.red[m][wv] = lo;
                sh.red[4 + m][wv] = hi;
                sh.red[8 + m][wv] = wt;
            }
        }
        __syncthreads();
        if (threadIdx.x < 12) {
            double v = sh.red[threadIdx.x][0];
            for (int w = 1; w < PT_T / 64; w++) v += sh.red[threadIdx.x][w];
            bs.base[bs.patch + 12 * lb + threadIdx.x] = v;
        }
    }
    if (!mine) return;
    int i = line, j = p;
    int b = bidx(B, i, j), cap = S.cap;
    size_t k = (size_t)j * g.nx + i;
    double as = Ls.alpha[k], ae = Le.alpha[k];
    double u2[4] = {0, 0, 0, 0};
    if (c.has)
        for (int m = 0; m < 4; m++) u2[m] = c.u1[m] + lam * ((sh.phi[m][x][cx] - sh.phi[m][x + 1][cx]) + W[m]);
    int gone = 0;
    if (as > 0.0 && ae == 0.0) {
        gone = 1;
    } else if (ae > 0.0 && c.has) {
        double r = u2[0], e = u2[3];
        if (!(r > 0.0) || !(e - 0.5 * (u2[1] * u2[1] + u2[2] * u2[2]) / r > 0.0)) {
            gone = 2;
            atomicAdd(ncollapse, 1u);
        }
    }
    for (int m = 0; m < 4; m++) S.U2[m * cap + b] = u2[m];
    S.gone[b] = (int8_t)gone;
}

// Content (conserved amounts) that is present but not an admissible gas state.
__device__ __forceinline__ bool inadmissible_content(const double* u) {
    if (u[0] == 0.0 && u[1] == 0.0 && u[2] == 0.0 && u[3] == 0.0) return false;
    double r = u[0];
    return !(r > 0.0) || !(u[3] - 0.5 * (u[1] * u[1] + u[2] * u[2]) / r > 0.0);
}

// Number of recipients of emptied box cell (ci, cj) in a round whose flags are `fl`: its
// face neighbours with end volume whose flag is 0 (not emptied, not bad), else such
// neighbours among all eight (cells outside the box have flag 0).
__device__ __forceinline__ int recipient_count(const Grid& g, const Level& Le, const Box& B, const int8_t* fl,
                                               int ci, int cj) {
    int nr = 0;
    for (int pass = 0; pass < 2 && nr == 0; pass++) {
        int cnt = pass == 0 ? 4 : 8;
        for (int q = 0; q < cnt; q++) {
            int ii = ci + c_d8[q][0], jj = cj + c_d8[q][1];
            if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny) continue;
            int8_t fk = B.has(ii, jj) ? fl[bidx(B, ii, jj)] : (int8_t)0;
            if (Le.alpha[(size_t)jj * g.nx + ii] > 0.0 && fk == 0) nr++;
        }
    }
    return nr;
}

// Covering (Eqs. massDeficitEquation, cutCellCoverDonation): each emptied cell's residual
// goes to its face neighbours that stay fluid (else its eight neighbours) in proportion to
// their end volume.  Gathered per recipient in increasing order of the emptied cell.
// want_lost: lost[] gets the residual of this thread's cell when it is emptied and has no
// recipient (it leaves the grid's totals); lost[] is left as it is otherwise.
template <typename R>
__device__ void cover(const Grid& g, const SweepJob& J, const Stage& S, int t, double (&lost)[4],
                      bool want_lost = false) {
    const Level& Le = J.Le;
    const Box& B = J.B;
    R* Uout = (R*)J.Uout;
    if (t >= B.w() * B.h()) return;
    int i = B.i0 + t % B.w(), j = B.j0 + t / B.w();
    int b = bidx(B, i, j), cap = S.cap;
    size_t nc = (size_t)g.nx * g.ny, k = (size_t)j * g.nx + i;
    double acc[4] = {0, 0, 0, 0};
    // the cell's own values and its neighbours' emptied flags, loaded together (neighbour
    // indices clamped into the box; the ones outside it are skipped below)
    int8_t gone_b = S.gone[b];
    double u2[4];
#pragma unroll
    for (int m = 0; m < 4; m++) u2[m] = S.U2[m * cap + b];
    double aer = Le.alpha[k];
    if (want_lost && gone_b && recipient_count(g, Le, B, S.gone, i, j) == 0)
        for (int m = 0; m < 4; m++) lost[m] = u2[m];
    unsigned gn = 0u;  // bit q: neighbour q (row-major in the 3 x 3 block) was emptied
#pragma unroll
    for (int q = 0; q < 9; q++) {
        int ci = min(max(i + q % 3 - 1, B.i0), B.i1 - 1), cj = min(max(j + q / 3 - 1, B.j0), B.j1 - 1);
        if (S.gone[bidx(B, ci, cj)]) gn |= 1u << q;
    }
    if (!gone_b) {
        for (int m = 0; m < 4; m++) acc[m] = u2[m];
        if (aer > 0.0) {
            for (int dj = -1; dj <= 1; dj++)
                for (int di = -1; di <= 1; di++) {
                    if (di == 0 && dj == 0) continue;
                    int ci = i + di, cj = j + dj;
                    if (!B.has(ci, cj)) continue;
                    int cb = bidx(B, ci, cj);
                    if (!((gn >> ((dj + 1) * 3 + (di + 1))) & 1u)) continue;
                    // recipients of the emptied cell (ci, cj)
                    int rec[8], nr = 0;
                    for (int pass = 0; pass < 2 && nr == 0; pass++) {
                        int cnt = pass == 0 ? 4 : 8;
                        for (int q = 0; q < cnt; q++) {
                            int ii = ci + c_d8[q][0], jj = cj + c_d8[q][1];
                            if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny) continue;
                            size_t kk = (size_t)jj * g.nx + ii;
                            bool gk = B.has(ii, jj) ? S.gone[bidx(B, ii, jj)] != 0 : false;
                            if (Le.alpha[kk] > 0.0 && !gk) rec[nr++] = (int)kk;
                        }
                    }
                    bool mine = false;
                    double den = 0.0;
                    for (int q = 0; q < nr; q++) {
                        den += Le.alpha[rec[q]];
                        mine |= rec[q] == (int)k;
                    }
                    if (!mine) continue;
                    double wgt = aer / den;
                    for (int m = 0; m < 4; m++) acc[m] += wgt * S.U2[m * cap + cb];
                }
        }
    }
    for (int m = 0; m < 4; m++) {
        Uout[m * nc + k] = (R)acc[m];
        S.U1[m * cap + b] = acc[m];
    }
    int8_t f = gone_b ? 2 : 0;
    if (!f && aer > 0.0 && inadmissible_content(acc)) {
        f = 1;
        atomicAdd(&S.nbad[0], 1u);
    }
    S.f1[b] = f;
}

// Collapse after covering (reading R28), one round: every cell flagged bad (content left
// that is not an admissible gas state) moves its content to its face neighbours that stay
// fluid and are neither bad nor emptied (else its eight neighbours), weighted by alpha_e;
// all bad cells of the round move at once, gathered per recipient in increasing order of
// the bad cell.  Round 0 flags the cells still bad for round 1; round 1 reports any cell
// still bad (status bit 2).  Both rounds return at once when the previous stage found no
// bad cell.
// want_lost: the content of a bad cell without recipients is added to lost[].
template <typename R>
__device__ void fix(const Grid& g, const SweepJob& J, const Stage& S, int round, unsigned int* ncollapse,
                    unsigned int* status, int t, double (&lost)[4], bool want_lost = false) {
    const Level& Le = J.Le;
    const Box& B = J.B;
    R* Uout = (R*)J.Uout;
    // content ping-pongs U1 -> Q -> U_out through the two rounds
    const double* Xin = round == 0 ? S.U1 : S.Q;
    const int8_t* fin = round == 0 ? S.f1 : S.f2;
    double* Xout = S.Q;
    int8_t* fout = S.f2;
    // the counter is read past the L1 cache: round 1 of a one-block launch reads what
    // round 0 counted with atomics in the same launch
    if (__hip_atomic_load(&S.nbad[round], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) return;
    if (t >= B.w() * B.h()) return;
    int i = B.i0 + t % B.w(), j = B.j0 + t / B.w();
    int b = bidx(B, i, j), cap = S.cap;
    size_t nc = (size_t)g.nx * g.ny, k = (size_t)j * g.nx + i;
    int8_t f = fin[b];
    double acc[4] = {0, 0, 0, 0};
    if (f == 1) {
        atomicAdd(ncollapse, 1u);
        if (want_lost && recipient_count(g, Le, B, fin, i, j) == 0)
            for (int m = 0; m < 4; m++) lost[m] += Xin[m * cap + b];
    } else {
        for (int m = 0; m < 4; m++) acc[m] = Xin[m * cap + b];
        double aer = Le.alpha[k];
        if (f == 0 && aer > 0.0) {
            for (int dj = -1; dj <= 1; dj++)
                for (int di = -1; di <= 1; di++) {
                    if (di == 0 && dj == 0) continue;
                    int ci = i + di, cj = j + dj;
                    if (!B.has(ci, cj)) continue;
                    int cb = bidx(B, ci, cj);
                    if (fin[cb] != 1) continue;
                    int rec[8], nr = 0;
                    for (int pass = 0; pass < 2 && nr == 0; pass++) {
                        int cnt = pass == 0 ? 4 : 8;
                        for (int q = 0; q < cnt; q++) {
                            int ii = ci + c_d8[q][0], jj = cj + c_d8[q][1];
                            if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny) continue;
                            size_t kk = (size_t)jj * g.nx + ii;
                            int8_t fk = B.has(ii, jj) ? fin[bidx(B, ii, jj)] : (int8_t)0;
                            if (Le.alpha[kk] > 0.0 && fk == 0) rec[nr++] = (int)kk;
                        }
                    }
                    bool mine = false;
                    double den = 0.0;
                    for (int q = 0; q < nr; q++) {
                        den += Le.alpha[rec[q]];
                        mine |= rec[q] == (int)k;
                    }
                    if (!mine) continue;
                    double wgt = aer / den;
                    for (int m = 0; m < 4; m++) acc[m] += wgt * Xin[m * cap + cb];
                }
        }
    }
    for (int m = 0; m < 4; m++) Uout[m * nc + k] = (R)acc[m];
    bool still = f == 0 && Le.alpha[k] > 0.0 && inadmissible_content(acc);
    if (round == 0) {
        for (int m = 0; m < 4; m++) Xout[m * cap + b] = acc[m];
        int8_t fo = f != 0 ? 2 : 0;
        if (still) {
            fo = 1;
            atomicAdd(&S.nbad[1], 1u);
        }
        fout[b] = fo;
    } else if (still) {
        atomicOr(status, 2u);
    }
}

// ------------------------------------------------------------------ dense sweeps
// Regular cells outside the sweep box: plain MUSCL-Hancock + HLLC update, U streamed once
// (read U_in, write U_out).  Both kernels are templated on the tile shape, chosen per grid
// by the tile tuner.

// Conservative update of a regular cell from its two face fluxes (fused in FP32).
template <typename T>
__device__ __forceinline__ T update(T q, T lam, T flo, T fhi) {
    if constexpr (sizeof(T) == 4) return __builtin_fmaf(lam, flo - fhi, q);
    return q + lam * (flo - fhi);
}

// Ghost-cell source index along a line of n cells (two layers; zero gradient or mirror).
__device__ __forceinline__ int ghost_src(int p, int n, int bclo, int bchi, bool& mir) {
    mir = false;
    int src = p;
    if (p < 0) {
        src = bclo == 1 ? -1 - p : 0;
        mir = bclo == 1;
    } else if (p >= n) {
        src = bchi == 1 ? 2 * n - 1 - p : n - 1;
        mir = bchi == 1;
    }
    return src < 0 ? 0 : (src >= n ? n - 1 : src);
}

// x-sweep: a block covers DX_OUT = 240 cells of RB consecutive rows.  Each of its four
// wavefronts takes 60 of them plus a two-cell halo each side (one lane per cell) and
// passes the neighbours' states, evolved face states and face fluxes between lanes by
// shuffles: no LDS and no barriers, so the wavefronts of a block never wait for each other
// (the halo lanes repeat 4 of every 64 cells' reconstructions).  The next row is loaded
// while the current one is computed.
constexpr int DX_T = 256;
constexpr int DX_WOUT = WAVE - 4;                // cells a wavefront writes
constexpr int DX_OUT = (DX_T / WAVE) * DX_WOUT;  // cells a block writes per row

template <int RB>
__host__ __device__ constexpr int dense_x_blocks(int nx, int ny) {
    return ((nx + DX_OUT - 1) / DX_OUT) * ((ny + RB - 1) / RB);
}

template <typename T>
__host__ __device__ constexpr size_t dense_x_lds() { return 0; }  // lane shuffles, no LDS

// Maximum of a per-lane bit-pattern pair over the wavefront (every lane gets it).
__device__ __forceinline__ void wave_max_pair(unsigned long long& bx, unsigned long long& by) {
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long ox = __shfl_xor(bx, off, 64), oy = __shfl_xor(by, off, 64);
        bx = ox > bx ? ox : bx;
        by = oy > by ? oy : by;
    }
}

// Dense tiles fold their speed maxima into this many shared slot pairs per member (tile lb
// into pair lb mod NSPD) with atomic maxima; the block that combines them resets them to
// zero, so between steps every slot holds zero.  The maximum does not depend on the order.
constexpr int NSPD = 256;

// Block maximum of a per-thread bit-pattern pair, written by thread 0 to out[0..1] (a
// block's own slot), or merged into them with atomic maxima (atomic: a shared slot).
// Every thread of the block calls it.
__device__ __forceinline__ void block_max_to(unsigned long long bx, unsigned long long by, unsigned long long* out,
                                             bool atomic = false) {
    __shared__ unsigned long long sx_[16], sy_[16];
    wave_max_pair(bx, by);
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sx_[w] = bx;
        sy_[w] = by;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < (int)(blockDim.x >> 6); q++) {
            bx = sx_[q] > bx ? sx_[q] : bx;
            by = sy_[q] > by ? sy_[q] : by;
        }
        if (atomic) {
            atomicMax(out, bx);
            atomicMax(out + 1, by);
        } else {
            out[0] = bx;
            out[1] = by;
        }
    }
    __syncthreads();
}

// Running maxima of the regular cells' speeds a dense tile writes, merged into the block's
// shared slot pair as FP64 bit patterns.  FP32 states keep 32-bit patterns until the flush (one
// integer maximum per step of the wavefront reduction instead of a 64-bit compare and two
// selects); the flushed pair equals the maximum of speed_bits over the same cells.
template <typename R>
struct SpeedMax {
    unsigned long long x = 0ull, y = 0ull;
    __device__ __forceinline__ void add(const R u[4], double gam) {
        unsigned long long bx, by;
        speed_bits(u, 1.0, gam, bx, by);
        x = bx > x ? bx : x;
        y = by > y ? by : y;
    }
    __device__ __forceinline__ void flush(unsigned long long* out) { block_max_to(x, y, out, true); }
};
template <>
struct SpeedMax<float> {
    unsigned x = 0u, y = 0u;
    __device__ __forceinline__ void add(const float u[4], double gam) {
        if (!(u[0] > 0.0f)) return;  // no gas: speed 0
        unsigned bx, by;
        speed_bits32(u, (float)gam, bx, by);
        x = max(x, bx);
        y = max(y, by);
    }
    __device__ __forceinline__ void flush(unsigned long long* out) {
        __shared__ unsigned sx_[16], sy_[16];
        for (int off = 32; off > 0; off >>= 1) {
            x = max(x, (unsigned)__shfl_xor((int)x, off, 64));
            y = max(y, (unsigned)__shfl_xor((int)y, off, 64));
        }
        int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            sx_[w] = x;
            sy_[w] = y;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int q = 1; q < (int)(blockDim.x >> 6); q++) {
                x = max(x, sx_[q]);
                y = max(y, sy_[q]);
            }
            atomicMax(out, bits32_to_64(x));
            atomicMax(out + 1, bits32_to_64(y));
        }
        __syncthreads();
    }
};

// lds: unused (kept for the callers that share a tile loop with LDS-staged kernels); cfl:
// when not null, the maxima of the written cells' speeds are merged into the slot pair
// (lb mod NSPD) of cfl; bud: when not null, the budget slots (the fluxes through the
// domain's low and high x-faces of the block's rows).  Every thread of the block calls it.
template <typename R, typename T, int RB>
__device__ __forceinline__ void dense_x(const Grid& g, const R* __restrict__ U_, R* __restrict__ Uout_, Box B, T lam,
                                        int lb, T* lds, unsigned long long* cfl, double* bud = nullptr) {
    (void)lds;  // the x-sweep exchanges values by lane shuffles
    const gmem<R>* __restrict__ U = to_global(U_);
    gmem<R>* __restrict__ Uout = to_global(Uout_);
    SpeedMax<R> sm;
    int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
    int nx = g.nx, ny = g.ny;
    int gx = (nx + DX_OUT - 1) / DX_OUT;
    int i = (lb % gx) * DX_OUT + wv * DX_WOUT - 2 + lane;
    int j0 = (lb / gx) * RB;
    size_t nc = (size_t)nx * ny;
    bool mir;
    int src = ghost_src(i, nx, g.bc[0], g.bc[1], mir);
    bool writer = lane >= 2 && lane < WAVE - 2 && i >= 0 && i < nx;
    bool colbox = i >= B.i0 && i < B.i1;
    T gam = (T)g.gamma;
    // budget: the threads of columns 0 and nx - 1 record the fluxes through the domain's
    // low and high faces of each row (zero for rows whose cell the box phases update)
    bool bedge = bud && writer && (i == 0 || i == nx - 1);
    if (bud && lb == 0 && tid == 0) bud[0] = (double)(2 * ny);
    T qn[4];
    {
        size_t kk = (size_t)j0 * nx + src;
#pragma unroll
        for (int m = 0; m < 4; m++) qn[m] = (T)U[m * nc + kk];
    }
    for (int r = 0; r < RB; r++) {
        int j = j0 + r;
        if (j >= ny) break;  // uniform over the block
        T q[4];
#pragma unroll
        for (int m = 0; m < 4; m++) q[m] = qn[m];
        if (r + 1 < RB && j + 1 < ny) {
            size_t kk = (size_t)(j + 1) * nx + src;
#pragma unroll
            for (int m = 0; m < 4; m++) qn[m] = (T)U[m * nc + kk];
        }
        if (mir) q[1] = -q[1];
        // lane l holds cell i: its reconstruction needs cells i - 1 and i + 1 (lanes 0 and
        // 63 get their own values, unused); face i - 1/2 needs cell i - 1's evolved right
        // state; the update needs face i + 1/2's flux from lane l + 1
        T qm[4], qp[4], el[4], er[4], erl[4], F[4], Fr[4];
#pragma unroll
        for (int m = 0; m < 4; m++) {
            qm[m] = __shfl_up(q[m], 1, WAVE);
            qp[m] = __shfl_down(q[m], 1, WAVE);
        }
        muscl<T, 0>(qm, q, qp, true, lam, gam, el, er);
#pragma unroll
        for (int m = 0; m < 4; m++) erl[m] = __shfl_up(er[m], 1, WAVE);
        hllc<T, 0>(erl, el, gam, F);
#pragma unroll
        for (int m = 0; m < 4; m++) Fr[m] = __shfl_down(F[m], 1, WAVE);
        if (writer && !(colbox && j >= B.j0 && j < B.j1)) {
            size_t k = (size_t)j * nx + i;
            R un[4];
#pragma unroll
            for (int m = 0; m < 4; m++) un[m] = (R)update(q[m], lam, F[m], Fr[m]);
#pragma unroll
            for (int m = 0; m < 4; m++) Uout[m * nc + k] = un[m];
            if (cfl) sm.add(un, g.gamma);
        }
        if (bedge) {
            bool upd = !(colbox && j >= B.j0 && j < B.j1);
            if (i == 0)
#pragma unroll
                for (int m = 0; m < 4; m++) bud[BS_DENSE + 4 * (2 * j) + m] = upd ? (double)F[m] : 0.0;
            if (i == nx - 1)
#pragma unroll
                for (int m = 0; m < 4; m++) bud[BS_DENSE + 4 * (2 * j + 1) + m] = upd ? (double)Fr[m] : 0.0;
        }
    }
    if (cfl) sm.flush(cfl + 2 * (lb % NSPD));
}

// y-sweep: a block covers 64 columns x TR rows.  The tile and its two-row halos (TR + 4
// rows, each a coalesced 64-wide access per component) are staged in LDS; then, as in the
// x-sweep, every cell's reconstruction, every face's flux and every cell's update is
// computed once, in three phases separated by barriers (rows spread over the four
// wavefronts).  The face fluxes reuse the staged states' LDS space.
template <typename T, int TR>
struct DenseYTile {
    static constexpr int ROWS = TR + 4;  // staged rows: tile rows 0 .. TR+3 (outputs 2 .. TR+1)
    static constexpr int ITS = (TR + 2 + 3) / 4;  // reconstructed rows 1 .. TR+2 per wavefront
    static constexpr size_t lds_bytes = (size_t)(ROWS + TR + 3) * 64 * 4 * sizeof(T);
};

template <int TR>
__host__ __device__ constexpr int dense_y_blocks(int nx, int ny) {
    return ((nx + 63) / 64) * ((ny + TR - 1) / TR);
}

template <typename R, typename T, int TR>
__device__ __forceinline__ void dense_y(const Grid& g, const R* __restrict__ U_, R* __restrict__ Uout_, Box B, T lam,
                                        int lb, T* lds, unsigned long long* cfl, double* bud = nullptr) {
    const gmem<R>* __restrict__ U = to_global(U_);
    gmem<R>* __restrict__ Uout = to_global(Uout_);
    using Tile = DenseYTile<T, TR>;
    constexpr int ROWS = Tile::ROWS, ITS = Tile::ITS;
    // staged states, then face fluxes (row r: face below cell r); evolved states at the
    // upper face of each cell
    T(*sq)[ROWS][64] = reinterpret_cast<T(*)[ROWS][64]>(lds);
    T(*ser)[TR + 3][64] = reinterpret_cast<T(*)[TR + 3][64]>(lds + 4 * ROWS * 64);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int nx = g.nx, ny = g.ny;
    int gx = (nx + 63) / 64;
    int i = (lb % gx) * 64 + lane;
    int jt = (lb / gx) * TR;  // grid row of tile row 2
    size_t nc = (size_t)nx * ny;
    int ic = i < nx ? i : nx - 1;
    for (int r = w; r < ROWS; r += 4) {
        bool mir;
        int src = ghost_src(jt - 2 + r, ny, g.bc[2], g.bc[3], mir);
        size_t k = (size_t)src * nx + ic;
        T v[4];
#pragma unroll
        for (int m = 0; m < 4; m++) v[m] = (T)U[m * nc + k];
        if (mir) v[2] = -v[2];
#pragma unroll
        for (int m = 0; m < 4; m++) sq[m][r][lane] = v[m];
    }
    __syncthreads();
    T gam = (T)g.gamma;
    T qc[ITS][4], el[ITS][4];
#pragma unroll
    for (int it = 0; it < ITS; it++) {
        int r = 1 + w + 4 * it;
        if (r > TR + 2) break;
        T qm[4], qp[4], er[4];
#pragma unroll
        for (int m = 0; m < 4; m++) {
            qm[m] = sq[m][r - 1][lane];
            qc[it][m] = sq[m][r][lane];
            qp[m] = sq[m][r + 1][lane];
        }
        muscl<T, 1>(qm, qc[it], qp, true, lam, gam, el[it], er);
#pragma unroll
        for (int m = 0; m < 4; m++) ser[m][r][lane] = er[m];
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ITS; it++) {
        int r = 1 + w + 4 * it;
        if (r > TR + 2) break;
        if (r < 2) continue;
        T erl[4], F[4];
#pragma unroll
        for (int m = 0; m < 4; m++) erl[m] = ser[m][r - 1][lane];
        hllc<T, 1>(erl, el[it], gam, F);
#pragma unroll
        for (int m = 0; m < 4; m++) sq[m][r][lane] = F[m];
    }
    __syncthreads();
    SpeedMax<R> sm;
    bool colbox = i >= B.i0 && i < B.i1;
    if (bud && lb == 0 && threadIdx.x == 0) bud[0] = (double)(2 * nx);
#pragma unroll
    for (int it = 0; it < ITS; it++) {
        int r = 1 + w + 4 * it;
        if (r > TR + 1) break;
        if (r < 2) continue;
        int jj = jt + r - 2;
        if (bud && i < nx && (jj == 0 || jj == ny - 1)) {
            // budget: the fluxes through the domain's low and high faces of column i (zero
            // when the box phases update that cell)
            bool upd = !(colbox && jj >= B.j0 && jj < B.j1);
            if (jj == 0)
#pragma unroll
                for (int m = 0; m < 4; m++) bud[BS_DENSE + 4 * (2 * i) + m] = upd ? (double)sq[m][r][lane] : 0.0;
            if (jj == ny - 1)
#pragma unroll
                for (int m = 0; m < 4; m++)
                    bud[BS_DENSE + 4 * (2 * i + 1) + m] = upd ? (double)sq[m][r + 1][lane] : 0.0;
        }
        if (i >= nx || jj >= ny || (colbox && jj >= B.j0 && jj < B.j1)) continue;
        size_t k = (size_t)jj * nx + i;
        R un[4];
#pragma unroll
        for (int m = 0; m < 4; m++) un[m] = (R)update(qc[it][m], lam, sq[m][r][lane], sq[m][r + 1][lane]);
#pragma unroll
        for (int m = 0; m < 4; m++) Uout[m * nc + k] = un[m];
        if (cfl) sm.add(un, g.gamma);
    }
    if (cfl) sm.flush(cfl + 2 * (lb % NSPD));
    __syncthreads();  // the caller may reuse the LDS for its next tile
}

// y-sweep, column walk: a block covers 256 columns x RW rows, and each thread walks its
// column down the block's rows with every state it needs in registers (no LDS, no
// barriers): the RW + 4 states of its column are loaded first, all in flight at once; then
// per row r the reconstruction of row r+1, the flux at the face between rows r and r+1 and
// the update of row r.  Each block computes RW + 2 reconstructions and RW + 1 fluxes per
// column, and every value with the same operations as the tiled sweep above, so the two
// give identical results.
constexpr int DYC_T = 256;

template <int RW>
__host__ __device__ constexpr int dense_yc_blocks(int nx, int ny) {
    return ((nx + DYC_T - 1) / DYC_T) * ((ny + RW - 1) / RW);
}

template <typename R, typename T, int RW>
__device__ __forceinline__ void dense_yc(const Grid& g, const R* __restrict__ U_, R* __restrict__ Uout_, Box B,
                                         T lam, int lb, unsigned long long* cfl, double* bud = nullptr) {
    const gmem<R>* __restrict__ U = to_global(U_);
    gmem<R>* __restrict__ Uout = to_global(Uout_);
    int nx = g.nx, ny = g.ny;
    int gx = (nx + DYC_T - 1) / DYC_T;
    int i = (lb % gx) * DYC_T + (int)threadIdx.x;
    int j0 = (lb / gx) * RW;  // grid row of the block's first output row
    size_t nc = (size_t)nx * ny;
    int ic = i < nx ? i : nx - 1;
    // q[k]: the state of row j0 - 2 + k (ghost rows mapped as in the tiled sweep)
    T q[RW + 4][4];
#pragma unroll
    for (int k = 0; k < RW + 4; k++) {
        bool mir;
        int src = ghost_src(j0 - 2 + k, ny, g.bc[2], g.bc[3], mir);
        size_t kk = (size_t)src * nx + ic;
#pragma unroll
        for (int m = 0; m < 4; m++) q[k][m] = (T)U[m * nc + kk];
        if (mir) q[k][2] = -q[k][2];
    }
    T gam = (T)g.gamma;
    T el[4], er[4], erp[4], flo[4], fhi[4];
    muscl<T, 1>(q[0], q[1], q[2], true, lam, gam, el, erp);  // row j0 - 1: its upper-face state
    muscl<T, 1>(q[1], q[2], q[3], true, lam, gam, el, er);   // row j0
    hllc<T, 1>(erp, el, gam, flo);                           // face below row j0
#pragma unroll
    for (int m = 0; m < 4; m++) erp[m] = er[m];
    SpeedMax<R> sm;
    bool colbox = i >= B.i0 && i < B.i1;
    if (bud && lb == 0 && threadIdx.x == 0) bud[0] = (double)(2 * nx);
#pragma unroll
    for (int r = 0; r < RW; r++) {
        int j = j0 + r;
        if (j >= ny) break;  // uniform over the block
        muscl<T, 1>(q[r + 2], q[r + 3], q[r + 4], true, lam, gam, el, er);  // row j + 1
        hllc<T, 1>(erp, el, gam, fhi);                                       // face above row j
        if (bud && i < nx && (j == 0 || j == ny - 1)) {
            // budget, as in the tiled sweep
            bool upd = !(colbox && j >= B.j0 && j < B.j1);
            if (j == 0)
#pragma unroll
                for (int m = 0; m < 4; m++) bud[BS_DENSE + 4 * (2 * i) + m] = upd ? (double)flo[m] : 0.0;
            if (j == ny - 1)
#pragma unroll
                for (int m = 0; m < 4; m++) bud[BS_DENSE + 4 * (2 * i + 1) + m] = upd ? (double)fhi[m] : 0.0;
        }
        if (i < nx && !(colbox && j >= B.j0 && j < B.j1)) {
            size_t k = (size_t)j * nx + i;
            R un[4];
#pragma unroll
            for (int m = 0; m < 4; m++) un[m] = (R)update(q[r + 2][m], lam, flo[m], fhi[m]);
#pragma unroll
            for (int m = 0; m < 4; m++) Uout[m * nc + k] = un[m];
            if (cfl) sm.add(un, g.gamma);
        }
#pragma unroll
        for (int m = 0; m < 4; m++) {
            flo[m] = fhi[m];
            erp[m] = er[m];
        }
    }
    if (cfl) sm.flush(cfl + 2 * (lb % NSPD));
}

}  // namespace cc
