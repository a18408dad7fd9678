// One directional sweep of the moving-boundary cut-cell method (Sec. 2.3.3-2.3.5):
// time-averaged apertures, states of cells that become fluid, wall Riemann problem and
// boundary flux, standard fluxes, stabilised shielded fluxes, conservative update and the
// covering of cells that become solid.
//
// Split of the work:
//   * dense kernels update every cell outside the sweep box (the bodies' region grown by
//     three cells): there all stencil cells are regular, so the plain MUSCL-Hancock/HLLC
//     update applies; they stream the state once (read U_in, write U_out);
//   * the box kernels (stage, swept apertures, wall, patch, cover) handle every cell of the
//     sweep box with the general cut-cell formulas, through box-local staging arrays.
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

// --------------------------------------------------------------- time-averaged apertures
// Exact average over the sweep of the aperture of a face normal to the sweep direction
// (Eq. timeAveragedBeta): the solid length integrated over the sweep is the area of the
// start polygon inside the strip swept across the face.
template <int D>
__global__ __launch_bounds__(256) void k_swept(Grid g, Level Ls, Level Le, Motion M, Box B, Stage S) {
    int t = wave_item(), lane = wave_lane();
    int fw = D == 0 ? B.w() + 1 : B.w(), fh = D == 0 ? B.h() : B.h() + 1;
    if (t >= fw * fh) return;
    int i = B.i0 + t % fw, j = B.j0 + t / fw;
    double bs = D == 0 ? beta_x(g, Ls, i, j) : beta_y(g, Ls, i, j);
    double be = D == 0 ? beta_x(g, Le, i, j) : beta_y(g, Le, i, j);
    double r;
    if (bs == 0.0 && be == 0.0) {
        r = 0.0;
    } else if (Ls.poly.m == 0) {
        r = 0.5 * (bs + be);
    } else {
        const Poly& P = Ls.poly;
        double X = vx_of(g, i), Y = vy_of(g, j);
        double h = D == 0 ? g.hx : g.hy, hf = D == 0 ? g.hy : g.hx;
        double Dd = D == 0 ? step_disp(M, 0, X, Y + 0.5 * g.hy) : step_disp(M, 1, X + 0.5 * g.hx, Y);
        if (!(fabs(Dd) > 1e-12 * h)) {
            r = 0.5 * (bs + be);
        } else {
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
            if (x0 + sw < P.xmin || x0 > P.xmax || y0 + sh < P.ymin || y0 > P.ymax) {
                r = 1.0;
            } else {
                double rs = wave_right_solid(P, x0, y0, sw, sh, lane);
                double a = wave_clip_area(P, x0, y0, sw, sh, rs, lane);
                r = 1.0 - a / (w * hf);
                if (r < 0.0) r = 0.0;
                if (r > 1.0) r = 1.0;
            }
        }
    }
    if (lane == 0) S.bt[fidx<D>(B, i, j)] = r;
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
            if (Ls.alpha[kk] > 0.0 && (double)U[kk] > 0.0) don[nd++] = (int)kk;
        }
    }
    return nd;
}

// States of the box cells before the sweep (Eqs. volumeWeighting, cutCellInitialisation,
// cutCellInitialisationDonorCellUpdate as read for exact time averages):
//   uncovered (alpha_s = 0 < alpha_e): state = donors' volume-weighted average, no content;
//   emptied (alpha_s > 0, no content): content sigma * sum(donor content);
//   donors of emptied cells keep the fraction (1 - sum sigma) of their content.
template <typename R>
__global__ void k_stage(Grid g, Level Ls, Level Le, const R* __restrict__ U, Box B, Stage S,
                        unsigned int* status) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) S.nbad[0] = S.nbad[1] = 0u;  // read by the collapse rounds at the sweep's end
    if (t >= B.w() * B.h()) return;
    int i = B.i0 + t % B.w(), j = B.j0 + t / B.w();
    size_t nc = (size_t)g.nx * g.ny, k = (size_t)j * g.nx + i;
    int cap = S.cap;
    double as = Ls.alpha[k], ae = Le.alpha[k];
    double u[4];
#pragma unroll
    for (int m = 0; m < 4; m++) u[m] = (double)U[m * nc + k];
    bool uncovered = as == 0.0 && ae > 0.0;
    bool emptied = as > 0.0 && ae > 0.0 && !(u[0] > 0.0);
    double q[4] = {0, 0, 0, 0};
    double u1[4] = {u[0], u[1], u[2], u[3]};
    int has = 0;
    if (uncovered || emptied) {
        int don[8];
        int nd = donors(g, Ls, U, i, j, don);
        if (nd == 0) {
            atomicOr(status, 1u);
        } else {
            double sa = 0.0;
            for (int qd = 0; qd < nd; qd++) sa += Ls.alpha[don[qd]];
            if (uncovered) {
                for (int m = 0; m < 4; m++) {
                    double su = 0.0;
                    for (int qd = 0; qd < nd; qd++) su += (double)U[m * nc + don[qd]];
                    q[m] = su / sa;
                }
                has = 1;
                u1[0] = u1[1] = u1[2] = u1[3] = 0.0;
            } else {
                double sig = as / (as + sa);
                for (int m = 0; m < 4; m++) {
                    double su = 0.0;
                    for (int qd = 0; qd < nd; qd++) su += (double)U[m * nc + don[qd]];
                    u1[m] = sig * su;
                }
            }
        }
    } else if (as > 0.0 && u[0] > 0.0) {
        // a live cell may donate to emptied neighbours (visited in increasing cell order)
        double take = 0.0;
        for (int dj = -1; dj <= 1; dj++)
            for (int di = -1; di <= 1; di++) {
                if (di == 0 && dj == 0) continue;
                int li = i + di, lj = j + dj;
                if (li < 0 || li >= g.nx || lj < 0 || lj >= g.ny) continue;
                size_t l = (size_t)lj * g.nx + li;
                double asl = Ls.alpha[l], ael = Le.alpha[l];
                if (!(asl > 0.0 && ael > 0.0 && !((double)U[l] > 0.0))) continue;
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
}

// ------------------------------------------------------------------ wall quantities
__device__ __forceinline__ bool cell_cut(const Grid& g, const Level& L, int i, int j) {
    double b[4] = {beta_x(g, L, i, j), beta_x(g, L, i + 1, j), beta_y(g, L, i, j), beta_y(g, L, i, j + 1)};
    int ones = 0, zeros = 0;
    for (int k = 0; k < 4; k++) {
        ones += b[k] == 1.0;
        zeros += b[k] == 0.0;
    }
    return ones != 4 && zeros != 4;
}

// Mean of the boundary crossing points on the cell's faces; cell centre if none.
__device__ void wall_point(const Grid& g, const Level& L, int i, int j, double* wx, double* wy) {
    double sx = 0.0, sy = 0.0;
    int n = 0;
    for (int e = 0; e < 4; e++) {
        double2 iv;
        double ox, oy, dx, dy;
        if (e < 2) {
            iv = L.fx[(size_t)j * (g.nx + 1) + i + e];
            ox = vx_of(g, i + e);
            oy = vy_of(g, j);
            dx = 0.0;
            dy = g.hy;
        } else {
            iv = L.fy[(size_t)(j + e - 2) * g.nx + i];
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

// Per box cell: wall flag, shielded volume, boundary flux F^B (advective part from the
// step's common boundary state, pressure part from this stage) and F^B - u_wall^d Q^B.
template <int D>
__global__ void k_wall(Grid g, Level Ls, Level Le, Motion M, Box B, Stage S, Common C, int first,
                       int32_t step_id) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B.w() * B.h()) return;
    int i = B.i0 + t % B.w(), j = B.j0 + t / B.w();
    int cap = S.cap, b = bidx(B, i, j);
    size_t nc = (size_t)g.nx * g.ny, k = (size_t)j * g.nx + i;
    double as = Ls.alpha[k], ae = Le.alpha[k];
    double ab = 0.5 * (as + ae);
    double bw, be, bs, bn;
    if (D == 0) {
        bw = S.bt[fidx<0>(B, i, j)];
        be = S.bt[fidx<0>(B, i + 1, j)];
        bs = 0.5 * (beta_y(g, Ls, i, j) + beta_y(g, Le, i, j));
        bn = 0.5 * (beta_y(g, Ls, i, j + 1) + beta_y(g, Le, i, j + 1));
    } else {
        bw = 0.5 * (beta_x(g, Ls, i, j) + beta_x(g, Le, i, j));
        be = 0.5 * (beta_x(g, Ls, i + 1, j) + beta_x(g, Le, i + 1, j));
        bs = S.bt[fidx<1>(B, i, j)];
        bn = S.bt[fidx<1>(B, i, j + 1)];
    }
    double Nx = (bw - be) * g.hy, Ny = (bs - bn) * g.hx;
    bool wall = ab > 0.0 && (Nx != 0.0 || Ny != 0.0);
    double fb[4] = {0, 0, 0, 0}, wv[4] = {0, 0, 0, 0}, ahat = 0.0;
    if (wall) {
        double nn = sqrt(Nx * Nx + Ny * Ny);
        double nxu = Nx / nn, nyu = Ny / nn;
        double wx, wy;
        bool cs = cell_cut(g, Ls, i, j), ce = cell_cut(g, Le, i, j);
        if (cs && ce) {
            double ax, ay, bx2, by2;
            wall_point(g, Ls, i, j, &ax, &ay);
            wall_point(g, Le, i, j, &bx2, &by2);
            wx = 0.5 * (ax + bx2);
            wy = 0.5 * (ay + by2);
        } else if (cs) {
            wall_point(g, Ls, i, j, &wx, &wy);
        } else {
            wall_point(g, Le, i, j, &wx, &wy);
        }
        double uwx = M.vx - M.thd * (wy - M.chy);
        double uwy = M.vy + M.thd * (wx - M.chx);
        double blo = D == 0 ? bw : bs, bhi = D == 0 ? be : bn;
        double mn = blo < bhi ? blo : bhi;
        double sh = fabs(bhi - blo);
        double ah = ab - mn;
        if (ah < 0.0) ah = 0.0;
        if (ah > sh) ah = sh;
        ahat = ah;
        if (S.has[b]) {
            double q[4];
            for (int m = 0; m < 4; m++) q[m] = S.Q[m * cap + b];
            double pst, rst;
            wall_riemann(q, nxu, nyu, uwx, uwy, g.gamma, &pst, &rst);
            double u = q[1] / q[0], v = q[2] / q[0];
            double un = u * nxu + v * nyu, wn = uwx * nxu + uwy * nyu;
            double usx = (u - un * nxu) + wn * nxu;
            double usy = (v - un * nyu) + wn * nyu;
            double qb[4];
            if (first || C.stamp[k] != step_id) {
                qb[0] = rst;
                qb[1] = rst * usx;
                qb[2] = rst * usy;
                qb[3] = pst / (g.gamma - 1.0) + 0.5 * rst * (usx * usx + usy * usy);
                if (first) {
                    for (int m = 0; m < 4; m++) C.qb[m * nc + k] = qb[m];
                    C.stamp[k] = step_id;
                }
            } else {
                for (int m = 0; m < 4; m++) qb[m] = C.qb[m * nc + k];
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

// ------------------------------------------------------------------ patch (box update)
struct CellData {
    double q[4];
    double u1[4];
    bool has;
};

// State of the cell at line position p (ghost cells beyond the domain: zero-gradient copy
// or mirror with negated normal momentum).
template <int D, typename R>
__device__ void fetch_cell(const Grid& g, const R* U, const Box& B, const Stage& S, int line, int p, int n,
                           CellData& c) {
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
    if (B.has(i, j)) {
        int b = bidx(B, i, j);
        c.has = S.has[b] != 0;
        for (int m = 0; m < 4; m++) {
            c.q[m] = S.Q[m * S.cap + b];
            c.u1[m] = S.U1[m * S.cap + b];
        }
    } else {
        size_t k = (size_t)j * g.nx + i;
        c.has = true;
        for (int m = 0; m < 4; m++) c.q[m] = c.u1[m] = (double)U[m * nc + k];
    }
    if (!c.has)
        for (int m = 0; m < 4; m++) c.q[m] = 0.0;
    if (mirror) c.q[1 + D] = -c.q[1 + D];
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
__device__ void fetch_wall(const Box& B, const Stage& S, int line, int p, int n, WallData& w) {
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
__device__ void face_phi(double bt, double btm, double btp, const double* er_l, const double* el_r, bool act,
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
__global__ void k_patch(Grid g, Level Ls, Level Le, const R* __restrict__ U, Box B, Stage S, double lam,
                        unsigned int* ncollapse) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
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
        for (int s = 0; s < 5; s++) fetch_cell<D>(g, U, B, S, line, p - 2 + s, n, c[s]);
        double el[3][4], er[3][4];
        for (int s = 1; s <= 3; s++) {
            if (!c[s].has) continue;
            bool ok = c[s - 1].has && c[s + 1].has;
            muscl<double, D>(c[s - 1].q, c[s].q, c[s + 1].q, ok, lam, gam, el[s - 1], er[s - 1]);
        }
        double bt[4];  // faces p-1, p, p+1, p+2
        for (int s = 0; s < 4; s++) bt[s] = face_bt<D>(B, S, line, p - 1 + s);
        WallData w[3];
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

// Content (conserved amounts) that is present but not an admissible gas state.
__device__ __forceinline__ bool inadmissible_content(const double* u) {
    if (u[0] == 0.0 && u[1] == 0.0 && u[2] == 0.0 && u[3] == 0.0) return false;
    double r = u[0];
    return !(r > 0.0) || !(u[3] - 0.5 * (u[1] * u[1] + u[2] * u[2]) / r > 0.0);
}

// Covering (Eqs. massDeficitEquation, cutCellCoverDonation): each emptied cell's residual
// goes to its face neighbours that stay fluid (else its eight neighbours) in proportion to
// their end volume.  Gathered per recipient in increasing order of the emptied cell.
template <typename R>
__global__ void k_cover(Grid g, Level Le, Box B, Stage S, R* __restrict__ Uout) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B.w() * B.h()) return;
    int i = B.i0 + t % B.w(), j = B.j0 + t / B.w();
    int b = bidx(B, i, j), cap = S.cap;
    size_t nc = (size_t)g.nx * g.ny, k = (size_t)j * g.nx + i;
    double acc[4] = {0, 0, 0, 0};
    if (!S.gone[b]) {
        for (int m = 0; m < 4; m++) acc[m] = S.U2[m * cap + b];
        double aer = Le.alpha[k];
        if (aer > 0.0) {
            for (int dj = -1; dj <= 1; dj++)
                for (int di = -1; di <= 1; di++) {
                    if (di == 0 && dj == 0) continue;
                    int ci = i + di, cj = j + dj;
                    if (!B.has(ci, cj)) continue;
                    int cb = bidx(B, ci, cj);
                    if (!S.gone[cb]) continue;
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
    int8_t f = S.gone[b] ? 2 : 0;
    if (!f && Le.alpha[k] > 0.0 && inadmissible_content(acc)) {
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
template <typename R>
__global__ void k_fix(Grid g, Level Le, Box B, Stage S, int round, const double* __restrict__ Xin,
                      const int8_t* __restrict__ fin, double* __restrict__ Xout, int8_t* __restrict__ fout,
                      R* __restrict__ Uout, unsigned int* ncollapse, unsigned int* status) {
    if (S.nbad[round] == 0u) return;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B.w() * B.h()) return;
    int i = B.i0 + t % B.w(), j = B.j0 + t / B.w();
    int b = bidx(B, i, j), cap = S.cap;
    size_t nc = (size_t)g.nx * g.ny, k = (size_t)j * g.nx + i;
    int8_t f = fin[b];
    double acc[4] = {0, 0, 0, 0};
    if (f == 1) {
        atomicAdd(ncollapse, 1u);
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
// x-sweep of regular cells: one thread per cell, 256-cell tiles with a two-cell halo on
// each side exchanged through LDS (slopes, evolved face states, face fluxes).
constexpr int DX_T = 256;
constexpr int DX_OUT = DX_T - 4;

template <typename R, typename T>
__global__ __launch_bounds__(DX_T) void k_dense_x(Grid g, const R* __restrict__ U, R* __restrict__ Uout, Box B,
                                                   T lam) {
    __shared__ T sq[4][DX_T];
    __shared__ T ser[4][DX_T];
    __shared__ T sf[4][DX_T];
    int tid = threadIdx.x;
    int j = blockIdx.y;
    int nx = g.nx;
    int i = blockIdx.x * DX_OUT - 2 + tid;
    size_t nc = (size_t)nx * g.ny;
    bool rowbox = j >= B.j0 && j < B.j1;
    // ghost mapping
    int src = i;
    bool mir = false;
    if (i < 0) {
        src = g.bc[0] == 1 ? -1 - i : 0;
        mir = g.bc[0] == 1;
    } else if (i >= nx) {
        src = g.bc[1] == 1 ? 2 * nx - 1 - i : nx - 1;
        mir = g.bc[1] == 1;
    }
    src = src < 0 ? 0 : (src >= nx ? nx - 1 : src);
    T q[4];
    size_t kk = (size_t)j * nx + src;
#pragma unroll
    for (int m = 0; m < 4; m++) q[m] = (T)U[m * nc + kk];
    if (mir) q[1] = -q[1];
#pragma unroll
    for (int m = 0; m < 4; m++) sq[m][tid] = q[m];
    __syncthreads();
    T el[4], er[4];
    if (tid >= 1 && tid < DX_T - 1) {
        T qm[4], qp[4];
#pragma unroll
        for (int m = 0; m < 4; m++) {
            qm[m] = sq[m][tid - 1];
            qp[m] = sq[m][tid + 1];
        }
        muscl<T, 0>(qm, q, qp, true, lam, (T)g.gamma, el, er);
#pragma unroll
        for (int m = 0; m < 4; m++) ser[m][tid] = er[m];
    }
    __syncthreads();
    if (tid >= 2 && tid < DX_T - 1) {
        T erl[4], F[4];
#pragma unroll
        for (int m = 0; m < 4; m++) erl[m] = ser[m][tid - 1];
        hllc<T, 0>(erl, el, (T)g.gamma, F);
#pragma unroll
        for (int m = 0; m < 4; m++) sf[m][tid] = F[m];
    }
    __syncthreads();
    if (tid >= 2 && tid < DX_T - 2 && i >= 0 && i < nx) {
        if (rowbox && i >= B.i0 && i < B.i1) return;
        size_t k = (size_t)j * nx + i;
#pragma unroll
        for (int m = 0; m < 4; m++) Uout[m * nc + k] = (R)(q[m] + lam * (sf[m][tid] - sf[m][tid + 1]));
    }
}

// y-sweep of regular cells: one thread per column segment of DY_ROWS rows, marching up
// the column with a register window (coalesced row-wise loads across the wavefront).
template <typename R, typename T>
__global__ __launch_bounds__(256) void k_dense_y(Grid g, const R* __restrict__ U, R* __restrict__ Uout, Box B,
                                                 T lam, int rows) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int nx = g.nx, ny = g.ny;
    if (i >= nx) return;
    int j0 = blockIdx.y * rows;
    int j1 = min(j0 + rows, ny);
    size_t nc = (size_t)nx * ny;
    bool colbox = i >= B.i0 && i < B.i1;
    auto load = [&](int jj, T* q) {
        int src = jj;
        bool mir = false;
        if (jj < 0) {
            src = g.bc[2] == 1 ? -1 - jj : 0;
            mir = g.bc[2] == 1;
        } else if (jj >= ny) {
            src = g.bc[3] == 1 ? 2 * ny - 1 - jj : ny - 1;
            mir = g.bc[3] == 1;
        }
        src = src < 0 ? 0 : (src >= ny ? ny - 1 : src);
        size_t k = (size_t)src * nx + i;
#pragma unroll
        for (int m = 0; m < 4; m++) q[m] = (T)U[m * nc + k];
        if (mir) q[2] = -q[2];
    };
    T qa[4], qb[4], qc[4];  // cells s-1, s, s+1
    load(j0 - 2, qa);
    load(j0 - 1, qb);
    T er_prev[4], F_prev[4], q_prev[4];
    for (int s = j0 - 1; s <= j1; s++) {
        load(s + 1, qc);
        T el[4], er[4];
        muscl<T, 1>(qa, qb, qc, true, lam, (T)g.gamma, el, er);
        if (s >= j0) {
            T F[4];
            hllc<T, 1>(er_prev, el, (T)g.gamma, F);  // face s, between cells s-1 and s
            if (s - 1 >= j0) {
                int jj = s - 1;
                if (!(colbox && jj >= B.j0 && jj < B.j1)) {
                    size_t k = (size_t)jj * nx + i;
#pragma unroll
                    for (int m = 0; m < 4; m++) Uout[m * nc + k] = (R)(q_prev[m] + lam * (F_prev[m] - F[m]));
                }
            }
#pragma unroll
            for (int m = 0; m < 4; m++) F_prev[m] = F[m];
        }
#pragma unroll
        for (int m = 0; m < 4; m++) {
            er_prev[m] = er[m];
            q_prev[m] = qb[m];
            qa[m] = qb[m];
            qb[m] = qc[m];
        }
    }
}

}  // namespace cc
