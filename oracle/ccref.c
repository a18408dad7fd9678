/*
 * ccref.c -- FP64 CPU oracle for one dimensionally split step of the moving-boundary
 * cut-cell method of Bennett, Nikiforakis & Klein (arXiv:1711.11361).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this file.
 * It exists so that tests, the smoke check and the CPU-baseline leg of the benchmark can
 * compare the GPU library against a plain, slow, obviously correct implementation.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Everything is FP64, evaluated in the written order (built with -ffp-contract=off, no
 * fast-math).  The whole grid is processed with plain loops; no blocking, no fusion.
 *
 * Where the paper is silent or garbled the reading used is stated at the point of use
 * (R-numbers refer to the list of readings kept with the design notes).
 *
 * Parity pins: closed forms (piston, normal shock, exact Riemann problem), brute-force
 * geometry, the static convex-combination identity, the free-stream identity, discrete
 * conservation and mirror symmetry are checked by the CPU test suite.  The generic moving
 * cut-cell values beyond those identities are "parity unpinned" (no printed values exist).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------------ */
/* Public structs (same field layout as the GPU library's config structs, written here  */
/* independently so that one ctypes description can feed both).                        */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    int32_t nx, ny;
    int32_t bc[4];     /* W, E, S, N : 0 transmissive (zero gradient), 1 reflective */
    int32_t precision; /* ignored by the oracle (always FP64) */
    int32_t options;   /* bit 0: axisymmetric about the x axis (y is the radius; reading R33) */
    double x_lo, x_hi, y_lo, y_hi;
    double gamma;
    double alpha_min;  /* cut cells with a smaller volume fraction count as solid (reading
                        * R19); 0 = none */
} ccref_config;

typedef struct {
    int32_t nverts;
    int32_t pad_;
    const double* verts; /* body frame, convex, counter-clockwise, (x,y) pairs */
    double ref_x, ref_y, theta0;
    double vx, vy;
    double pitch_amp, pitch_omega;
} ccref_body;

enum { FLUID = 0, SOLID = 1 };

/* Sweep record of the traced cell (ccref_trace): standard fluxes F of its low and high
 * faces (4 + 4), stabilised fluxes Phi of those faces (4 + 4), its boundary flux F^B (4),
 * its state Q (4), then alpha_s, alpha_e, the time-averaged apertures of its low and high
 * faces, the shielded volume, the wall flag and the state flag (7). */
#define TRACE_N 31

/* Several bodies (reading R30): the solid region is the union of up to CCREF_MAX_BODIES
 * closed convex polygons, each with its own prescribed motion.  Bodies must not meet
 * inside one face or one cell: a face with solid parts from two bodies, a cell with
 * solid area from two bodies, or a wall cell cut by one body at the sweep's start and by
 * another at its end sets status bit 4. */
#define CCREF_MAX_BODIES 4

typedef struct {
    int8_t* vcls;  /* (ny+1)*(nx+1) vertex classes */
    double* fx;    /* 2*ny*(nx+1) solid intervals of x-faces (face (i,j) between cells (i-1,j),(i,j)) */
    double* fy;    /* 2*(ny+1)*nx solid intervals of y-faces (face (i,j) between cells (i,j-1),(i,j)) */
    double* alpha; /* ny*nx volume fractions */
    int np;        /* posed polygons of this level (one per body) */
    double* poly[CCREF_MAX_BODIES];
    int m[CCREF_MAX_BODIES];
    int8_t* cbody; /* several bodies: the body cutting each cut cell, -1 elsewhere (else NULL) */
} level_t;

typedef struct {
    int m;              /* polygon vertex count, 0 = no body */
    double* bverts;     /* body-frame polygon */
    double ref_x, ref_y, theta0, vx, vy, amp, omega;
    double cosd, sind, c0x, c0y, c1x, c1y; /* rigid map of the current step */
} body_t;

typedef struct {
    ccref_config cfg;
    double hx, hy;
    int nb;             /* bodies (1 for a context without a body: B[0].m = 0) */
    body_t B[CCREF_MAX_BODIES];
    double* U;          /* 4*ny*nx conserved amount per unit CELL volume, planes rho,mx,my,E */
    level_t L[3];       /* level slots */
    int s0, sm, s1;     /* slots of level n, stage level, level n+1 */
    double t;           /* time of level n */
    int64_t step;       /* steps taken */
    int parity;         /* 0: x then y, 1: y then x */
    /* step-in-progress bookkeeping */
    int in_step, sweeps_done;
    double step_dt;
    /* cell state stored on the step's first sweep (advective boundary state, per cell) */
    double* Q0;
    int64_t* stamp0;
    /* budgets (accumulated over all sweeps) */
    double bnd[4], wall[4], lost[4];
    int status;
    int64_t ncollapse; /* cells emptied because their update was not admissible */
    /* test hooks: a cell whose sweep quantities the next sweeps record, and the record */
    int trace_i, trace_j;
    double trace[TRACE_N];
    /* oracle-only option: a cell that becomes fluid takes content from its donors as
     * printed (Eq. cutCellInitialisationDonorCellUpdate) instead of only a state (R13) */
    int uncover_moves_content;
} ccref_ctx;

/* ------------------------------------------------------------------------------------ */
/* Gas model: Euler equations with a perfect-gas equation of state (Sec. 2.1).          */
/* Q = (rho, rho u, rho v, E),  p = (gamma-1) (E - (mx^2+my^2)/(2 rho)).                */
/* ------------------------------------------------------------------------------------ */
static double pressure(const double q[4], double g) {
    return (g - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0]);
}

/* Physical flux in direction d (0 = x, 1 = y). */
static void euler_flux(const double q[4], int d, double g, double f[4]) {
    double p = pressure(q, g);
    int n = 1 + d, t = 2 - d;
    double un = q[n] / q[0];
    f[0] = q[n];
    f[n] = q[n] * un + p;
    f[t] = q[t] * un;
    f[3] = un * (q[3] + p);
}

/* HLLC flux (Toro's approximate Riemann solver, named in Sec. 2.3.5) with Davis wave-speed
 * estimates, in direction d.  ql is the state on the low side of the face. */
static void hllc(const double ql[4], const double qr[4], int d, double g, double f[4]) {
    int n = 1 + d, t = 2 - d;
    double rl = ql[0], rr = qr[0];
    double ul = ql[n] / rl, ur = qr[n] / rr;
    double pl = pressure(ql, g), pr = pressure(qr, g);
    double al = sqrt(g * pl / rl), ar = sqrt(g * pr / rr);
    double sl = fmin(ul - al, ur - ar);
    double sr = fmax(ul + al, ur + ar);
    double ss = (pr - pl + rl * ul * (sl - ul) - rr * ur * (sr - ur)) /
                (rl * (sl - ul) - rr * (sr - ur));
    if (0.0 <= sl) {
        euler_flux(ql, d, g, f);
    } else if (0.0 <= ss) {
        double fl[4], us[4];
        euler_flux(ql, d, g, fl);
        double c = rl * (sl - ul) / (sl - ss);
        us[0] = c;
        us[n] = c * ss;
        us[t] = c * (ql[t] / rl);
        us[3] = c * (ql[3] / rl + (ss - ul) * (ss + pl / (rl * (sl - ul))));
        for (int k = 0; k < 4; k++) f[k] = fl[k] + sl * (us[k] - ql[k]);
    } else if (0.0 <= sr) {
        double fr[4], us[4];
        euler_flux(qr, d, g, fr);
        double c = rr * (sr - ur) / (sr - ss);
        us[0] = c;
        us[n] = c * ss;
        us[t] = c * (qr[t] / rr);
        us[3] = c * (qr[3] / rr + (ss - ur) * (ss + pr / (rr * (sr - ur))));
        for (int k = 0; k < 4; k++) f[k] = fr[k] + sr * (us[k] - qr[k]);
    } else {
        euler_flux(qr, d, g, f);
    }
}

/* van Leer limiter (harmonic mean of the one-sided differences, zero at extrema). */
static double vanleer(double a, double b) {
    if (a * b > 0.0) return 2.0 * a * b / (a + b);
    return 0.0;
}

static int admissible(const double q[4], double g) {
    if (!(q[0] > 0.0)) return 0;
    return pressure(q, g) > 0.0;
}

/* MUSCL-Hancock reconstruction and half-step evolution of one cell (Sec. 2.3.5 end).
 * slope_ok: both stencil neighbours carry a state.  Outputs the evolved states at the
 * low face (el) and the high face (er) of the cell. */
static void muscl_cell(const double qm[4], const double q[4], const double qp[4], int slope_ok,
                       double lam, int d, double g, double el[4], double er[4]) {
    double dl[4] = {0, 0, 0, 0};
    if (slope_ok)
        for (int k = 0; k < 4; k++) dl[k] = vanleer(q[k] - qm[k], qp[k] - q[k]);
    for (int pass = 0; pass < 2; pass++) {
        double ql[4], qr[4], fl[4], fr[4];
        for (int k = 0; k < 4; k++) {
            ql[k] = q[k] - 0.5 * dl[k];
            qr[k] = q[k] + 0.5 * dl[k];
        }
        int ok = admissible(ql, g) && admissible(qr, g);
        if (ok) {
            euler_flux(ql, d, g, fl);
            euler_flux(qr, d, g, fr);
            for (int k = 0; k < 4; k++) {
                double c = 0.5 * lam * (fl[k] - fr[k]);
                el[k] = ql[k] + c;
                er[k] = qr[k] + c;
            }
            ok = admissible(el, g) && admissible(er, g);
        }
        if (ok || pass == 1) {
            if (!ok) { /* first-order fallback: no evolution needed for a flat profile */
                for (int k = 0; k < 4; k++) el[k] = er[k] = q[k];
            }
            return;
        }
        /* positivity fallback: drop the slope and redo */
        for (int k = 0; k < 4; k++) dl[k] = 0.0;
    }
}

/* ------------------------------------------------------------------------------------ */
/* Geometry of one level (Sec. 2.1: volume fractions; Sec. 2.2: face apertures).        */
/* The body is a convex polygon.  A level stores: for every grid vertex whether it lies */
/* in the closed polygon; for every face the solid part of the face segment, as a       */
/* parameter interval [lo, hi] measured from the face's low-index vertex; for every     */
/* cell the fluid volume fraction, from the exact clip of the polygon to the cell.      */
/* ------------------------------------------------------------------------------------ */
static double orient(const double* a, const double* b, double px, double py) {
    return (b[0] - a[0]) * (py - a[1]) - (b[1] - a[1]) * (px - a[0]);
}

typedef struct {
    int m;
    const double* v; /* posed polygon, CCW */
    double xmin, xmax, ymin, ymax;
} poly_t;

static void poly_init(poly_t* P, const double* v, int m) {
    P->m = m;
    P->v = v;
    P->xmin = P->ymin = INFINITY;
    P->xmax = P->ymax = -INFINITY;
    for (int k = 0; k < m; k++) {
        P->xmin = fmin(P->xmin, v[2 * k]);
        P->xmax = fmax(P->xmax, v[2 * k]);
        P->ymin = fmin(P->ymin, v[2 * k + 1]);
        P->ymax = fmax(P->ymax, v[2 * k + 1]);
    }
}

/* Closed-polygon membership: solid iff on or left of every edge (boundary is solid);
 * points outside the polygon's bounding box are fluid without testing. */
static int classify(const poly_t* P, double px, double py) {
    if (P->m == 0) return FLUID;
    if (px < P->xmin || px > P->xmax || py < P->ymin || py > P->ymax) return FLUID;
    for (int k = 0; k < P->m; k++) {
        const double* a = P->v + 2 * k;
        const double* b = P->v + 2 * ((k + 1) % P->m);
        if (orient(a, b, px, py) < 0.0) return FLUID;
    }
    return SOLID;
}

/* Solid part of the segment A->B (Cyrus-Beck clip against the polygon's half-planes).
 * Returns 1 and the parameter interval [lo, hi] if it has positive length. */
static int seg_clip(const poly_t* P, double ax, double ay, double bx, double by, double* lo,
                    double* hi) {
    double tl = 0.0, th = 1.0;
    for (int k = 0; k < P->m; k++) {
        const double* a = P->v + 2 * k;
        const double* b = P->v + 2 * ((k + 1) % P->m);
        double g0 = orient(a, b, ax, ay), g1 = orient(a, b, bx, by);
        if (g0 < 0.0 && g1 < 0.0) return 0;
        if (g0 >= 0.0 && g1 >= 0.0) continue;
        double t = g0 / (g0 - g1);
        if (g0 < 0.0) {
            if (t > tl) tl = t; /* entering */
        } else {
            if (t < th) th = t; /* leaving */
        }
    }
    if (!(tl < th)) return 0;
    *lo = tl;
    *hi = th;
    return 1;
}

/* Solid interval of the face from vertex A (class ca) to vertex B (class cb). */
static void face_interval(const poly_t* P, double ax, double ay, int ca, double bx, double by,
                          int cb, double* lo, double* hi) {
    *lo = 0.0;
    *hi = 0.0;
    if (P->m == 0) return;
    if (ca == SOLID && cb == SOLID) { /* convex body: the whole face is solid */
        *hi = 1.0;
        return;
    }
    if (fmax(ax, bx) < P->xmin || fmin(ax, bx) > P->xmax || fmax(ay, by) < P->ymin ||
        fmin(ay, by) > P->ymax)
        return; /* disjoint bounding boxes */
    double l, h;
    if (seg_clip(P, ax, ay, bx, by, &l, &h)) {
        *lo = l;
        *hi = h;
    }
}

/* Fluid fraction of a face from its solid interval. */
static double interval_beta(double lo, double hi) { return hi > lo ? 1.0 - (hi - lo) : 1.0; }

/* Area of the polygon clipped to the rectangle [ox, ox+w] x [oy, oy+h], computed in
 * coordinates relative to (ox, oy) by Sutherland-Hodgman clipping and the shoelace
 * formula.  b1, b2: scratch of 2*(m+8) doubles each. */
static double clip_area(const double* v, int m, double ox, double oy, double w, double h,
                        double* b1, double* b2) {
    int n = m;
    for (int k = 0; k < m; k++) {
        b1[2 * k] = v[2 * k] - ox;
        b1[2 * k + 1] = v[2 * k + 1] - oy;
    }
    double* in = b1;
    double* out = b2;
    for (int side = 0; side < 4 && n > 0; side++) {
        /* side 0: x >= 0, 1: x <= w, 2: y >= 0, 3: y <= h */
        int ax = side < 2 ? 0 : 1;
        double lim = side == 0 || side == 2 ? 0.0 : (side == 1 ? w : h);
        int keep_ge = side == 0 || side == 2;
        int no = 0;
        for (int k = 0; k < n; k++) {
            const double* S = in + 2 * ((k + n - 1) % n);
            const double* E = in + 2 * k;
            int sin_ = keep_ge ? S[ax] >= lim : S[ax] <= lim;
            int ein = keep_ge ? E[ax] >= lim : E[ax] <= lim;
            if (sin_ != ein) {
                double t = (lim - S[ax]) / (E[ax] - S[ax]);
                double I[2];
                I[ax] = lim;
                I[1 - ax] = S[1 - ax] + t * (E[1 - ax] - S[1 - ax]);
                out[2 * no] = I[0];
                out[2 * no + 1] = I[1];
                no++;
            }
            if (ein) {
                out[2 * no] = E[0];
                out[2 * no + 1] = E[1];
                no++;
            }
        }
        double* tmp = in;
        in = out;
        out = tmp;
        n = no;
    }
    double acc = 0.0;
    for (int k = 0; k < n; k++) {
        int k1 = (k + 1) % n;
        acc += in[2 * k] * in[2 * k1 + 1] - in[2 * k1] * in[2 * k + 1];
    }
    return 0.5 * acc;
}

static double vx_of(const ccref_ctx* c, int i) { return c->cfg.x_lo + (double)i * c->hx; }
static double vy_of(const ccref_ctx* c, int j) { return c->cfg.y_lo + (double)j * c->hy; }

#define VIDX(c, i, j) ((size_t)(j) * (size_t)((c)->cfg.nx + 1) + (size_t)(i))
#define BXIDX(c, i, j) ((size_t)(j) * (size_t)((c)->cfg.nx + 1) + (size_t)(i))
#define BYIDX(c, i, j) ((size_t)(j) * (size_t)(c)->cfg.nx + (size_t)(i))
#define CIDX(c, i, j) ((size_t)(j) * (size_t)(c)->cfg.nx + (size_t)(i))

static double beta_x(const ccref_ctx* c, const level_t* L, int i, int j) {
    size_t f = BXIDX(c, i, j);
    return interval_beta(L->fx[2 * f], L->fx[2 * f + 1]);
}
static double beta_y(const ccref_ctx* c, const level_t* L, int i, int j) {
    size_t f = BYIDX(c, i, j);
    return interval_beta(L->fy[2 * f], L->fy[2 * f + 1]);
}

/* A cell is cut when its four faces are neither all open nor all closed. */
static int cell_is_cut(const ccref_ctx* c, const level_t* L, int i, int j) {
    double b[4] = {beta_x(c, L, i, j), beta_x(c, L, i + 1, j), beta_y(c, L, i, j),
                   beta_y(c, L, i, j + 1)};
    int ones = 0, zeros = 0;
    for (int k = 0; k < 4; k++) {
        ones += b[k] == 1.0;
        zeros += b[k] == 0.0;
    }
    return ones != 4 && zeros != 4;
}

/* Wall point of a cut cell: the mean of the points where the body boundary crosses the
 * cell's faces (interval end points strictly inside a face); the cell centre if none. */
static void wall_point(const ccref_ctx* c, const level_t* L, int i, int j, double* wx,
                       double* wy) {
    double sx = 0.0, sy = 0.0;
    int n = 0;
    for (int e = 0; e < 4; e++) {
        const double* iv;
        double ox, oy, dx, dy;
        if (e < 2) { /* W, E x-faces: from vertex (i+e, j) upwards */
            iv = L->fx + 2 * BXIDX(c, i + e, j);
            ox = vx_of(c, i + e);
            oy = vy_of(c, j);
            dx = 0.0;
            dy = c->hy;
        } else { /* S, N y-faces: from vertex (i, j+e-2) rightwards */
            iv = L->fy + 2 * BYIDX(c, i, j + e - 2);
            ox = vx_of(c, i);
            oy = vy_of(c, j + e - 2);
            dx = c->hx;
            dy = 0.0;
        }
        if (!(iv[1] > iv[0])) continue;
        for (int q = 0; q < 2; q++) {
            double t = iv[q];
            if (t > 0.0 && t < 1.0) {
                sx += ox + t * dx;
                sy += oy + t * dy;
                n++;
            }
        }
    }
    if (n == 0) {
        *wx = vx_of(c, i) + 0.5 * c->hx;
        *wy = vy_of(c, j) + 0.5 * c->hy;
        return;
    }
    *wx = sx / (double)n;
    *wy = sy / (double)n;
}

/* Closed bounding boxes of polygon P and of the rectangle [x0, x1] x [y0, y1] are disjoint. */
static int rect_misses(const poly_t* P, double x0, double y0, double x1, double y1) {
    return P->m == 0 || x1 < P->xmin || x0 > P->xmax || y1 < P->ymin || y0 > P->ymax;
}

/* Solid interval of the face A->B with several bodies (reading R30): the one body whose
 * polygon meets the face in a segment of positive length (ends classified against that
 * body); *bad is set when two bodies do.  With one body: face_interval with the level's
 * vertex classes (ca, cb). */
static void face_interval_any(const poly_t* P, int np, double ax, double ay, int ca, double bx,
                              double by, int cb, double* lo, double* hi, int* bad) {
    if (np == 1) {
        face_interval(&P[0], ax, ay, ca, bx, by, cb, lo, hi);
        return;
    }
    *lo = 0.0;
    *hi = 0.0;
    int hits = 0;
    for (int b = 0; b < np; b++) {
        double l, h;
        face_interval(&P[b], ax, ay, classify(&P[b], ax, ay), bx, by, classify(&P[b], bx, by), &l, &h);
        if (h > l) {
            if (hits == 0) {
                *lo = l;
                *hi = h;
            }
            hits++;
        }
    }
    if (hits > 1) *bad = 1;
}

/* Body of cut cell (i, j) with several bodies: the first whose polygon covers part of the
 * cell (area[b] > 0), else the first that closes part of one of its faces, else 0. */
static int cell_body(const ccref_ctx* c, const poly_t* P, int np, const double* area, int i, int j) {
    for (int b = 0; b < np; b++)
        if (area[b] > 0.0) return b;
    double x0 = vx_of(c, i), x1 = vx_of(c, i + 1), y0 = vy_of(c, j), y1 = vy_of(c, j + 1);
    double seg[4][4] = {{x0, y0, x0, y1}, {x1, y0, x1, y1}, {x0, y0, x1, y0}, {x0, y1, x1, y1}};
    for (int b = 0; b < np; b++)
        for (int e = 0; e < 4; e++) {
            const double* q = seg[e];
            double l, h;
            face_interval(&P[b], q[0], q[1], classify(&P[b], q[0], q[1]), q[2], q[3],
                          classify(&P[b], q[2], q[3]), &l, &h);
            if (h > l) return b;
        }
    return 0;
}

/* Geometry of a level from np posed polygons (one per body). */
static void compute_level(ccref_ctx* c, const double* const* pv, const int* pm, int np, level_t* L) {
    int nx = c->cfg.nx, ny = c->cfg.ny;
    poly_t P[CCREF_MAX_BODIES];
    int mmax = 1;
    L->np = np;
    for (int b = 0; b < np; b++) {
        L->poly[b] = realloc(L->poly[b], sizeof(double) * 2 * (size_t)(pm[b] > 0 ? pm[b] : 1));
        if (pm[b] > 0) memcpy(L->poly[b], pv[b], sizeof(double) * 2 * (size_t)pm[b]);
        L->m[b] = pm[b];
        poly_init(&P[b], L->poly[b], pm[b]);
        if (pm[b] > mmax) mmax = pm[b];
    }
    int bad = 0;
    /* every loop below writes each item once from the level's inputs only: the rows may
     * run in any order (OpenMP build) with identical results */
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= ny; j++)
        for (int i = 0; i <= nx; i++) {
            int cls = FLUID;
            for (int b = 0; b < np && cls == FLUID; b++) cls = classify(&P[b], vx_of(c, i), vy_of(c, j));
            L->vcls[VIDX(c, i, j)] = (int8_t)cls;
        }
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i <= nx; i++) {
            size_t f = BXIDX(c, i, j);
            face_interval_any(P, np, vx_of(c, i), vy_of(c, j), L->vcls[VIDX(c, i, j)], vx_of(c, i),
                              vy_of(c, j + 1), L->vcls[VIDX(c, i, j + 1)], &L->fx[2 * f], &L->fx[2 * f + 1], &bad);
        }
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int j = 0; j <= ny; j++)
        for (int i = 0; i < nx; i++) {
            size_t f = BYIDX(c, i, j);
            face_interval_any(P, np, vx_of(c, i), vy_of(c, j), L->vcls[VIDX(c, i, j)], vx_of(c, i + 1),
                              vy_of(c, j), L->vcls[VIDX(c, i + 1, j)], &L->fy[2 * f], &L->fy[2 * f + 1], &bad);
        }
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int j = 0; j < ny; j++) {
        double* b1 = malloc(sizeof(double) * 2 * (size_t)(mmax + 8));
        double* b2 = malloc(sizeof(double) * 2 * (size_t)(mmax + 8));
        for (int i = 0; i < nx; i++) {
            double b[4] = {beta_x(c, L, i, j), beta_x(c, L, i + 1, j), beta_y(c, L, i, j),
                           beta_y(c, L, i, j + 1)};
            int ones = 0, zeros = 0;
            for (int k = 0; k < 4; k++) {
                ones += b[k] == 1.0;
                zeros += b[k] == 0.0;
            }
            double a;
            int body = -1;
            if (ones == 4) {
                a = 1.0;
            } else if (zeros == 4) {
                a = 0.0;
            } else {
                double s;
                if (np == 1) {
                    s = clip_area(L->poly[0], pm[0], vx_of(c, i), vy_of(c, j), c->hx, c->hy, b1, b2);
                } else {
                    /* several bodies: the solid area is the sum of the bodies' areas in the
                     * cell, at most one of which may be positive */
                    double ab[CCREF_MAX_BODIES];
                    int hits = 0;
                    s = 0.0;
                    for (int q = 0; q < np; q++) {
                        ab[q] = 0.0;
                        if (!rect_misses(&P[q], vx_of(c, i), vy_of(c, j), vx_of(c, i) + c->hx, vy_of(c, j) + c->hy))
                            ab[q] = clip_area(L->poly[q], pm[q], vx_of(c, i), vy_of(c, j), c->hx, c->hy, b1, b2);
                        hits += ab[q] > 0.0;
                        s += ab[q];
                    }
                    if (hits > 1) bad = 1;
                    body = cell_body(c, P, np, ab, i, j);
                }
                a = 1.0 - s / (c->hx * c->hy);
                if (a < 0.0) a = 0.0;
                if (a > 1.0) a = 1.0;
                if (a < c->cfg.alpha_min) a = 0.0; /* small-cell threshold (reading R19) */
            }
            L->alpha[CIDX(c, i, j)] = a;
            if (L->cbody) L->cbody[CIDX(c, i, j)] = (int8_t)body;
        }
        free(b1);
        free(b2);
    }
    if (bad) c->status |= 4;
}

/* ------------------------------------------------------------------------------------ */
/* Body pose and prescribed rigid motion.                                               */
/* theta(t) = theta0 + A sin(omega t), centre c(t) = ref + v t.                          */
/* ------------------------------------------------------------------------------------ */
static void pose(const ccref_ctx* c, int b, double t, double* out) {
    const body_t* B = &c->B[b];
    double th = B->theta0 + B->amp * sin(B->omega * t);
    double cs = cos(th), sn = sin(th);
    double cx = B->ref_x + B->vx * t, cy = B->ref_y + B->vy * t;
    for (int k = 0; k < B->m; k++) {
        double bx = B->bverts[2 * k], by = B->bverts[2 * k + 1];
        out[2 * k] = (cs * bx - sn * by) + cx;
        out[2 * k + 1] = (sn * bx + cs * by) + cy;
    }
}

/* Rigid-body velocity at point (x, y) at time t. */
static void body_velocity(const ccref_ctx* c, int b, double t, double x, double y, double* ux, double* uy) {
    const body_t* B = &c->B[b];
    double thd = B->amp * B->omega * cos(B->omega * t);
    double cx = B->ref_x + B->vx * t, cy = B->ref_y + B->vy * t;
    *ux = B->vx - thd * (y - cy);
    *uy = B->vy + thd * (x - cx);
}

/* ------------------------------------------------------------------------------------ */
/* Context management.                                                                  */
/* ------------------------------------------------------------------------------------ */
static int level_alloc(ccref_ctx* c, level_t* L) {
    size_t nx = c->cfg.nx, ny = c->cfg.ny;
    L->vcls = calloc((nx + 1) * (ny + 1), 1);
    L->fx = calloc(2 * ny * (nx + 1), sizeof(double));
    L->fy = calloc(2 * (ny + 1) * nx, sizeof(double));
    L->alpha = calloc(nx * ny, sizeof(double));
    L->np = 0;
    if (c->nb > 1) {
        L->cbody = malloc(nx * ny);
        if (L->cbody) memset(L->cbody, 0xff, nx * ny);
    }
    return L->vcls && L->fx && L->fy && L->alpha && (c->nb == 1 || L->cbody);
}

void ccref_destroy(ccref_ctx* c) {
    if (!c) return;
    for (int s = 0; s < 3; s++) {
        free(c->L[s].vcls);
        free(c->L[s].fx);
        free(c->L[s].fy);
        free(c->L[s].alpha);
        free(c->L[s].cbody);
        for (int b = 0; b < CCREF_MAX_BODIES; b++) free(c->L[s].poly[b]);
    }
    free(c->U);
    for (int b = 0; b < CCREF_MAX_BODIES; b++) free(c->B[b].bverts);
    free(c->Q0);
    free(c->stamp0);
    free(c);
}

/* A context with nbodies bodies (0 or NULL: none; several: reading R30, each with at
 * least three vertices). */
ccref_ctx* ccref_create_bodies(const ccref_config* cfg, const ccref_body* bodies, int nbodies) {
    if (cfg->nx < 1 || cfg->ny < 1 || !(cfg->x_hi > cfg->x_lo) || !(cfg->y_hi > cfg->y_lo)) return NULL;
    if (!(cfg->alpha_min >= 0.0 && cfg->alpha_min < 0.5)) return NULL;
    if (cfg->options & ~1 || ((cfg->options & 1) && !(cfg->y_lo >= 0.0))) return NULL;
    if (nbodies < 0 || nbodies > CCREF_MAX_BODIES || (nbodies > 0 && !bodies)) return NULL;
    for (int b = 0; nbodies > 1 && b < nbodies; b++)
        if (bodies[b].nverts < 3) return NULL;
    ccref_ctx* c = calloc(1, sizeof(ccref_ctx));
    if (!c) return NULL;
    c->cfg = *cfg;
    c->hx = (cfg->x_hi - cfg->x_lo) / (double)cfg->nx;
    c->hy = (cfg->y_hi - cfg->y_lo) / (double)cfg->ny;
    c->nb = nbodies > 1 ? nbodies : 1;
    for (int b = 0; b < nbodies; b++) {
        const ccref_body* body = &bodies[b];
        body_t* B = &c->B[b];
        B->m = body->nverts > 0 ? body->nverts : 0;
        if (B->m == 0) continue;
        B->bverts = malloc(sizeof(double) * 2 * B->m);
        memcpy(B->bverts, body->verts, sizeof(double) * 2 * B->m);
        B->ref_x = body->ref_x;
        B->ref_y = body->ref_y;
        B->theta0 = body->theta0;
        B->vx = body->vx;
        B->vy = body->vy;
        B->amp = body->pitch_amp;
        B->omega = body->pitch_omega;
    }
    size_t nc = (size_t)cfg->nx * cfg->ny;
    c->U = calloc(4 * nc, sizeof(double));
    c->Q0 = calloc(4 * nc, sizeof(double));
    c->stamp0 = malloc(nc * sizeof(int64_t));
    for (size_t k = 0; k < nc; k++) c->stamp0[k] = -1;
    int ok = c->U && c->Q0 && c->stamp0;
    for (int s = 0; s < 3; s++) ok = ok && level_alloc(c, &c->L[s]);
    if (!ok) {
        ccref_destroy(c);
        return NULL;
    }
    c->s0 = 0;
    c->sm = 1;
    c->s1 = 2;
    c->trace_i = c->trace_j = -1;
    return c;
}

ccref_ctx* ccref_create(const ccref_config* cfg, const ccref_body* body) {
    return ccref_create_bodies(cfg, body, body ? 1 : 0);
}

/* The bodies posed at time t (x coordinates at tx, y coordinates at ty: the stage level of
 * a split step mixes the two, reading R11) and the level's geometry from them. */
static void level_posed(ccref_ctx* c, double tx, double ty, level_t* L) {
    double* pv[CCREF_MAX_BODIES];
    int pm[CCREF_MAX_BODIES];
    for (int b = 0; b < c->nb; b++) {
        int m = c->B[b].m;
        pm[b] = m;
        pv[b] = malloc(sizeof(double) * 2 * (m > 0 ? m : 1));
        double* py = malloc(sizeof(double) * 2 * (m > 0 ? m : 1));
        pose(c, b, tx, pv[b]);
        pose(c, b, ty, py);
        for (int k = 0; k < m; k++) pv[b][2 * k + 1] = py[2 * k + 1];
        free(py);
    }
    compute_level(c, (const double* const*)pv, pm, c->nb, L);
    for (int b = 0; b < c->nb; b++) free(pv[b]);
}

static void level_at_time(ccref_ctx* c, double t, level_t* L) { level_posed(c, t, t, L); }

/* Initial state from primitive fields (rho, u, v, p) given per cell: U = alpha * Q. */
int ccref_set_prim(ccref_ctx* c, const double* prim, double t0) {
    size_t nc = (size_t)c->cfg.nx * c->cfg.ny;
    double g = c->cfg.gamma;
    c->t = t0;
    c->step = 0;
    c->parity = 0;
    c->in_step = 0;
    c->status = 0;
    c->ncollapse = 0;
    for (int k = 0; k < 4; k++) c->bnd[k] = c->wall[k] = c->lost[k] = 0.0;
    for (size_t k = 0; k < nc; k++) c->stamp0[k] = -1; /* step numbers restart */
    level_at_time(c, t0, &c->L[c->s0]);
    for (size_t k = 0; k < nc; k++) {
        double r = prim[k], u = prim[nc + k], v = prim[2 * nc + k], p = prim[3 * nc + k];
        double a = c->L[c->s0].alpha[k];
        double q[4] = {r, r * u, r * v, p / (g - 1.0) + 0.5 * r * (u * u + v * v)};
        for (int m = 0; m < 4; m++) c->U[m * nc + k] = a * q[m];
    }
    return 0;
}

/* Resume the clock: time t after `step` completed split steps, so that the next step's
 * sweep order (x then y after an even number of steps, y then x after an odd one) and the
 * level-n geometry (body posed at t) are those of an uninterrupted run.  The state is left
 * as it is; set it afterwards with ccref_set_u. */
int ccref_set_clock(ccref_ctx* c, double t, int64_t step) {
    if (step < 0) return 1;
    c->t = t;
    c->step = step;
    c->parity = (int)(step & 1);
    c->in_step = 0;
    for (size_t k = 0; k < (size_t)c->cfg.nx * c->cfg.ny; k++) c->stamp0[k] = -1;
    level_at_time(c, t, &c->L[c->s0]);
    return 0;
}

int ccref_set_u(ccref_ctx* c, const double* U) {
    memcpy(c->U, U, sizeof(double) * 4 * (size_t)c->cfg.nx * c->cfg.ny);
    return 0;
}
int ccref_get_u(const ccref_ctx* c, double* U) {
    memcpy(U, c->U, sizeof(double) * 4 * (size_t)c->cfg.nx * c->cfg.ny);
    return 0;
}
/* Primitive fields (rho,u,v,p) of the level-n state; cells with alpha = 0 give zeros. */
int ccref_get_prim(const ccref_ctx* c, double* prim) {
    size_t nc = (size_t)c->cfg.nx * c->cfg.ny;
    const double* al = c->L[c->s0].alpha;
    for (size_t k = 0; k < nc; k++) {
        double q[4] = {0, 0, 0, 0};
        int live = al[k] > 0.0 && c->U[k] > 0.0;
        if (live)
            for (int m = 0; m < 4; m++) q[m] = c->U[m * nc + k] / al[k];
        if (live) {
            prim[k] = q[0];
            prim[nc + k] = q[1] / q[0];
            prim[2 * nc + k] = q[2] / q[0];
            prim[3 * nc + k] = pressure(q, c->cfg.gamma);
        } else {
            prim[k] = prim[nc + k] = prim[2 * nc + k] = prim[3 * nc + k] = 0.0;
        }
    }
    return 0;
}

double ccref_time(const ccref_ctx* c) { return c->t; }
int64_t ccref_steps(const ccref_ctx* c) { return c->step; }
int ccref_parity(const ccref_ctx* c) { return c->parity; }
int ccref_status(const ccref_ctx* c) { return c->status; }
int64_t ccref_collapses(const ccref_ctx* c) { return c->ncollapse; }

/* Logical level names: 0 = level n, 1 = stage level, 2 = level n+1. */
static int slot_of(const ccref_ctx* c, int which) {
    return which == 0 ? c->s0 : which == 1 ? c->sm : which == 2 ? c->s1 : -1;
}

/* Posed polygon of body 0 at time t into out (2*m doubles); returns m. */
int ccref_pose(const ccref_ctx* c, double t, double* out) {
    pose(c, 0, t, out);
    return c->B[0].m;
}

/* Geometry of an arbitrary posed polygon into slot (for geometry tests). */
int ccref_geometry_poly(ccref_ctx* c, const double* posed, int m, int which) {
    int slot = slot_of(c, which);
    if (slot < 0) return 1;
    compute_level(c, &posed, &m, 1, &c->L[slot]);
    return 0;
}
/* Geometry of the body posed at time t into slot. */
int ccref_geometry(ccref_ctx* c, double t, int which) {
    int slot = slot_of(c, which);
    if (slot < 0) return 1;
    level_at_time(c, t, &c->L[slot]);
    return 0;
}

/* Copy a level out: vertex classes, volume fractions, x- and y-face apertures. */
int ccref_geometry_dump(const ccref_ctx* c, int which, int8_t* vcls, double* alpha, double* bx,
                        double* by) {
    size_t nx = c->cfg.nx, ny = c->cfg.ny;
    int s = slot_of(c, which);
    if (s < 0) return 1;
    const level_t* L = &c->L[s];
    if (vcls) memcpy(vcls, L->vcls, (nx + 1) * (ny + 1));
    if (alpha) memcpy(alpha, L->alpha, sizeof(double) * nx * ny);
    if (bx)
        for (size_t f = 0; f < ny * (nx + 1); f++) bx[f] = interval_beta(L->fx[2 * f], L->fx[2 * f + 1]);
    if (by)
        for (size_t f = 0; f < (ny + 1) * nx; f++) by[f] = interval_beta(L->fy[2 * f], L->fy[2 * f + 1]);
    return 0;
}

/* Cut cells of a level (neither all four faces open nor all four closed), as linear
 * indices j*nx + i in increasing order; *n receives their number.  out: nx*ny entries. */
int ccref_cut_list(const ccref_ctx* c, int which, int32_t* out, int32_t* n) {
    int s = slot_of(c, which);
    if (s < 0) return 1;
    int k = 0;
    for (int j = 0; j < c->cfg.ny; j++)
        for (int i = 0; i < c->cfg.nx; i++)
            if (cell_is_cut(c, &c->L[s], i, j)) out[k++] = (int32_t)CIDX(c, i, j);
    *n = k;
    return 0;
}

/* Solid intervals of the faces of a level (2 doubles per face). */
int ccref_face_intervals(const ccref_ctx* c, int which, double* fx, double* fy) {
    size_t nx = c->cfg.nx, ny = c->cfg.ny;
    int s = slot_of(c, which);
    if (s < 0) return 1;
    if (fx) memcpy(fx, c->L[s].fx, sizeof(double) * 2 * ny * (nx + 1));
    if (fy) memcpy(fy, c->L[s].fy, sizeof(double) * 2 * (ny + 1) * nx);
    return 0;
}

/* Wall point (mean of crossing points) of cell (i,j) of a level; returns 0 if not cut. */
int ccref_wall_point(const ccref_ctx* c, int which, int i, int j, double* wxy) {
    int slot = slot_of(c, which);
    if (slot < 0) return 0;
    const level_t* L = &c->L[slot];
    if (!cell_is_cut(c, L, i, j)) return 0;
    wall_point(c, L, i, j, wxy, wxy + 1);
    return 1;
}

/* ------------------------------------------------------------------------------------ */
/* Global time step (Sec. 4: a global step from the regular cell size; formula: reading */
/* R17): dt = C min(hx/Sx, hy/Sy), S = max(|u|+a) over live cells and |u_wall| over the  */
/* body's vertices.                                                                     */
/* ------------------------------------------------------------------------------------ */
int ccref_wave_speeds(const ccref_ctx* c, double* sxy) {
    size_t nc = (size_t)c->cfg.nx * c->cfg.ny;
    const double* al = c->L[c->s0].alpha;
    double g = c->cfg.gamma, sx = 0.0, sy = 0.0;
    for (size_t k = 0; k < nc; k++) {
        if (!(al[k] > 0.0) || !(c->U[k] > 0.0)) continue; /* solid or emptied */
        double q[4];
        for (int m = 0; m < 4; m++) q[m] = c->U[m * nc + k] / al[k];
        double u = q[1] / q[0], v = q[2] / q[0];
        double a = sqrt(g * pressure(q, g) / q[0]);
        sx = fmax(sx, fabs(u) + a);
        sy = fmax(sy, fabs(v) + a);
    }
    for (int b = 0; b < c->nb; b++) {
        int m = c->B[b].m;
        if (m == 0) continue;
        double* pv = malloc(sizeof(double) * 2 * m);
        pose(c, b, c->t, pv);
        for (int k = 0; k < m; k++) {
            double ux, uy;
            body_velocity(c, b, c->t, pv[2 * k], pv[2 * k + 1], &ux, &uy);
            sx = fmax(sx, fabs(ux));
            sy = fmax(sy, fabs(uy));
        }
        free(pv);
    }
    sxy[0] = sx;
    sxy[1] = sy;
    return 0;
}

double ccref_cfl_dt(const ccref_ctx* c, double cfl) {
    double s[2];
    ccref_wave_speeds(c, s);
    return cfl * fmin(c->hx / s[0], c->hy / s[1]);
}

/* Conservation totals: sum of U times the cell area, per component. */
int ccref_totals(const ccref_ctx* c, double* out4) {
    size_t nc = (size_t)c->cfg.nx * c->cfg.ny;
    double area = c->hx * c->hy;
    for (int m = 0; m < 4; m++) {
        double s = 0.0;
        for (size_t k = 0; k < nc; k++) s += c->U[m * nc + k];
        out4[m] = s * area;
    }
    return 0;
}

/* Budget accumulated since set_prim: domain-boundary fluxes, wall pressure terms and
 * residuals that found no recipient (all times cell area). */
int ccref_budget(const ccref_ctx* c, double* bnd4, double* wall4, double* lost4) {
    for (int k = 0; k < 4; k++) {
        if (bnd4) bnd4[k] = c->bnd[k];
        if (wall4) wall4[k] = c->wall[k];
        if (lost4) lost4[k] = c->lost[k];
    }
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* One sweep (Sec. 2.3.3-2.3.5, Eqs. Klein2shieldedFluxMethod2, ModifiedBoundaryFlux-    */
/* Method2, Klein2DtotalfluxaMethod2, Klein2DcompleteMovingMethod2a/b, volumeWeighting, */
/* cutCellInitialisation, cutCellInitialisationDonorCellUpdate, massDeficitEquation,    */
/* cutCellCoverDonation).                                                               */
/* ------------------------------------------------------------------------------------ */

/* Wall Riemann problem along the unit normal n (pointing into the solid) between the cut
 * cell's state and its mirror image moving with the wall (Eq. riemann_wallvel), solved
 * with the same HLLC/Davis machinery as the faces (reading R9).  Returns p*, rho*. */
static void wall_riemann(const double q[4], double nxu, double nyu, double wx, double wy, double g,
                         double* pst, double* rst) {
    double r = q[0];
    double u = q[1] / r, v = q[2] / r;
    double p = pressure(q, g);
    double a = sqrt(g * p / r);
    double un = u * nxu + v * nyu;
    double wn = wx * nxu + wy * nyu;
    double ul = un, ur = 2.0 * wn - un;
    double sl = fmin(ul - a, ur - a);
    double sr = fmax(ul + a, ur + a);
    double ss = (p - p + r * ul * (sl - ul) - r * ur * (sr - ur)) / (r * (sl - ul) - r * (sr - ur));
    double ps = p + r * (sl - ul) * (ss - ul);
    double rs = r * (sl - ul) / (sl - ss);
    if (ps < 0.0) ps = 0.0; /* reading: no negative wall pressure from the linearised star state */
    *pst = ps;
    *rst = rs;
}

typedef struct {
    double as, ae, ab;   /* alpha at start, end, time average */
    int wall;            /* wall cell in this sweep */
    double nx, ny;       /* unit wall normal (into solid) */
    double uwx, uwy;     /* wall velocity */
    double pst;          /* wall pressure p* of this sweep */
    double usx, usy;     /* boundary velocity of this sweep */
    double qb[4];        /* common boundary state (advective part) */
    double fb[4];        /* boundary flux in the sweep direction */
    double ahat;         /* shielded volume fraction */
} cellinfo;

/* Linear-in-time average of a face aperture (used for the faces across the sweep
 * direction, which only enter the wall normal and the shielded volume). */
static double beta_avg_x(const ccref_ctx* c, const level_t* Ls, const level_t* Le, int i, int j) {
    return 0.5 * (beta_x(c, Ls, i, j) + beta_x(c, Le, i, j));
}
static double beta_avg_y(const ccref_ctx* c, const level_t* Ls, const level_t* Le, int i, int j) {
    return 0.5 * (beta_y(c, Ls, i, j) + beta_y(c, Le, i, j));
}

/* Displacement, in direction d, of the point at (x, y) of body b under the step's rigid
 * map M(X) = R(theta1 - theta0) (X - c0) + c1. */
static double step_disp(const ccref_ctx* c, int b, int d, double x, double y) {
    const body_t* B = &c->B[b];
    double dx = x - B->c0x, dy = y - B->c0y;
    if (d == 0) return ((B->cosd * dx - B->sind * dy) + B->c1x) - x;
    return ((B->sind * dx + B->cosd * dy) + B->c1y) - y;
}

/* Exact time average over the sweep of the aperture of a face normal to the sweep
 * direction (Eq. timeAveragedBeta): during the sweep the level-s polygon moves by D along
 * the sweep direction, so the solid length integrated over the sweep equals the area of
 * the polygon inside the strip of width |D| swept across the face. */
static double swept_beta(const ccref_ctx* c, const level_t* Ls, const level_t* Le,
                         const poly_t* Ps, int dir, int i, int j, double* b1, double* b2) {
    double bs = dir == 0 ? beta_x(c, Ls, i, j) : beta_y(c, Ls, i, j);
    double be = dir == 0 ? beta_x(c, Le, i, j) : beta_y(c, Le, i, j);
    if (bs == 0.0 && be == 0.0) return 0.0; /* covered throughout (convex body) */
    if (Ps->m == 0) return 0.5 * (bs + be);
    double X = vx_of(c, i), Y = vy_of(c, j);
    double h = dir == 0 ? c->hx : c->hy, hf = dir == 0 ? c->hy : c->hx;
    double D = dir == 0 ? step_disp(c, 0, 0, X, Y + 0.5 * c->hy) : step_disp(c, 0, 1, X + 0.5 * c->hx, Y);
    if (!(fabs(D) > 1e-12 * h)) return 0.5 * (bs + be);
    double w = fabs(D);
    double x0, y0, sw, sh;
    if (dir == 0) {
        x0 = D > 0.0 ? X - D : X;
        y0 = Y;
        sw = w;
        sh = hf;
    } else {
        x0 = X;
        y0 = D > 0.0 ? Y - D : Y;
        sw = hf;
        sh = w;
    }
    if (x0 + sw < Ps->xmin || x0 > Ps->xmax || y0 + sh < Ps->ymin || y0 > Ps->ymax) return 1.0;
    double a = clip_area(Ps->v, Ps->m, x0, y0, sw, sh, b1, b2);
    double bt = 1.0 - a / (w * hf);
    if (bt < 0.0) bt = 0.0;
    if (bt > 1.0) bt = 1.0;
    return bt;
}

/* The same with several bodies (reading R30): each body moves by its own displacement D_b
 * at the face's midpoint, so the face's solid length integrated over the sweep is the sum
 * over the bodies of area(P_b at level s inside the strip of width |D_b|) / |D_b|, times
 * the sweep's duration; a body that does not move there contributes the average of its
 * solid fractions of the face at the two levels. */
static double seg_solid(const poly_t* P, double ax, double ay, double bx, double by) {
    double l, h;
    face_interval(P, ax, ay, classify(P, ax, ay), bx, by, classify(P, bx, by), &l, &h);
    return h > l ? h - l : 0.0;
}
static double swept_beta_bodies(const ccref_ctx* c, const level_t* Ls, const level_t* Le,
                                const poly_t* Ps, const poly_t* Pe, int dir, int i, int j,
                                double* b1, double* b2) {
    double bs = dir == 0 ? beta_x(c, Ls, i, j) : beta_y(c, Ls, i, j);
    double be = dir == 0 ? beta_x(c, Le, i, j) : beta_y(c, Le, i, j);
    if (bs == 0.0 && be == 0.0) return 0.0; /* covered throughout (bodies apart) */
    double X = vx_of(c, i), Y = vy_of(c, j);
    double h = dir == 0 ? c->hx : c->hy, hf = dir == 0 ? c->hy : c->hx;
    double ax = X, ay = Y, fx = dir == 0 ? X : X + c->hx, fy = dir == 0 ? Y + c->hy : Y;
    double solid = 0.0;
    for (int b = 0; b < Ls->np; b++) {
        double D = dir == 0 ? step_disp(c, b, 0, X, Y + 0.5 * c->hy) : step_disp(c, b, 1, X + 0.5 * c->hx, Y);
        if (!(fabs(D) > 1e-12 * h)) {
            solid += 0.5 * (seg_solid(&Ps[b], ax, ay, fx, fy) + seg_solid(&Pe[b], ax, ay, fx, fy));
            continue;
        }
        double w = fabs(D);
        double x0, y0, sw, sh;
        if (dir == 0) {
            x0 = D > 0.0 ? X - D : X;
            y0 = Y;
            sw = w;
            sh = hf;
        } else {
            x0 = X;
            y0 = D > 0.0 ? Y - D : Y;
            sw = hf;
            sh = w;
        }
        if (rect_misses(&Ps[b], x0, y0, x0 + sw, y0 + sh)) continue;
        solid += clip_area(Ps[b].v, Ps[b].m, x0, y0, sw, sh, b1, b2) / (w * hf);
    }
    double bt = 1.0 - solid;
    if (bt < 0.0) bt = 0.0;
    if (bt > 1.0) bt = 1.0;
    return bt;
}

int ccref_sweep(ccref_ctx* c, int dir, double dt) {
    int nx = c->cfg.nx, ny = c->cfg.ny;
    size_t nc = (size_t)nx * ny;
    double g = c->cfg.gamma;
    if (!c->in_step || c->sweeps_done > 1) return 1;
    int first = c->sweeps_done == 0;
    int want = first ? c->parity : 1 - c->parity;
    if (dir != want) return 1;
    const level_t* Ls = &c->L[first ? c->s0 : c->sm];
    const level_t* Le = &c->L[first ? c->sm : c->s1];
    double h = dir == 0 ? c->hx : c->hy;
    double lam = dt / h;
    double area = c->hx * c->hy;
    double thalf = c->t + 0.5 * c->step_dt;

    /* --- 1. cells without a usable state at the start of the sweep (Eqs. volumeWeighting,
     *        cutCellInitialisation, cutCellInitialisationDonorCellUpdate; readings R13, R27):
     *        * uncovered (alpha_s = 0 < alpha_e): the state used for its fluxes is the
     *          volume-weighted average of its donors; no content moves, because the exact
     *          time-averaged apertures already bring the swept-in fluid through its faces;
     *        * emptied by a collapse (alpha_s > 0, no content): refilled with content taken
     *          from its donors by the volume weighting.
     *        Donors: 4-neighbours with alpha_s > 0 and content, else 8-neighbours.  All
     *        donations are simultaneous (computed from the pre-donation values). --- */
    double* U1 = malloc(sizeof(double) * 4 * nc);
    memcpy(U1, c->U, sizeof(double) * 4 * nc);
    double* take = calloc(nc, sizeof(double));
    double* Qinit = calloc(4 * nc, sizeof(double)); /* states of uncovered cells */
    unsigned char* uncov = calloc(nc, 1);
    static const int d8[8][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}, {-1, -1}, {1, -1}, {-1, 1}, {1, 1}};
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            size_t l = CIDX(c, i, j);
            double asl = Ls->alpha[l], ael = Le->alpha[l];
            int uncovered = asl == 0.0 && ael > 0.0;
            int emptied = asl > 0.0 && ael > 0.0 && !(c->U[l] > 0.0);
            if (!uncovered && !emptied) continue;
            int don[8], nd = 0;
            for (int pass = 0; pass < 2 && nd == 0; pass++) {
                int cnt = pass == 0 ? 4 : 8;
                for (int q = 0; q < cnt; q++) {
                    int ii = i + d8[q][0], jj = j + d8[q][1];
                    if (ii < 0 || ii >= nx || jj < 0 || jj >= ny) continue;
                    size_t kk = CIDX(c, ii, jj);
                    if (Ls->alpha[kk] > 0.0 && c->U[kk] > 0.0) don[nd++] = (int)kk;
                }
            }
            if (nd == 0) {
                c->status |= 1; /* cell without donors */
                continue;
            }
            double sa = 0.0;
            for (int q = 0; q < nd; q++) sa += Ls->alpha[don[q]];
            if (uncovered && c->uncover_moves_content) {
                /* as printed: the new cell's content is the fraction sigma of its donors'
                 * content, sigma = alpha_e / (alpha_e + sum alpha_s of the donors), which the
                 * donors give up; its state is that content over its new volume */
                double sig = ael / (ael + sa);
                uncov[l] = 2;
                for (int m = 0; m < 4; m++) {
                    double su = 0.0;
                    for (int q = 0; q < nd; q++) su += c->U[m * nc + don[q]];
                    U1[m * nc + l] = sig * su;
                }
                for (int q = 0; q < nd; q++) take[don[q]] += sig;
            } else if (uncovered) {
                uncov[l] = 1;
                for (int m = 0; m < 4; m++) {
                    double su = 0.0;
                    for (int q = 0; q < nd; q++) su += c->U[m * nc + don[q]];
                    Qinit[m * nc + l] = su / sa;
                }
            } else {
                double sig = asl / (asl + sa);
                for (int m = 0; m < 4; m++) {
                    double su = 0.0;
                    for (int q = 0; q < nd; q++) su += c->U[m * nc + don[q]];
                    U1[m * nc + l] = sig * su;
                }
                for (int q = 0; q < nd; q++) take[don[q]] += sig;
            }
        }
    for (size_t k = 0; k < nc; k++)
        if (take[k] > 0.0)
            for (int m = 0; m < 4; m++) U1[m * nc + k] = c->U[m * nc + k] * (1.0 - take[k]);
    free(take);

    /* --- 2. time-averaged apertures of the faces normal to the sweep direction --- */
    size_t nfd = dir == 0 ? (size_t)ny * (nx + 1) : (size_t)(ny + 1) * nx;
    double* btd = malloc(sizeof(double) * nfd);
    {
        poly_t Ps[CCREF_MAX_BODIES], Pe[CCREF_MAX_BODIES];
        int mmax = 1;
        for (int b = 0; b < Ls->np; b++) {
            poly_init(&Ps[b], Ls->poly[b], Ls->m[b]);
            poly_init(&Pe[b], Le->poly[b], Le->m[b]);
            if (Ls->m[b] > mmax) mmax = Ls->m[b];
        }
        int rows = dir == 0 ? ny : ny + 1;
        int multi = Ls->np > 1;
#pragma omp parallel for schedule(static)
        for (int j = 0; j < rows; j++) {
            double* b1 = malloc(sizeof(double) * 2 * (size_t)(mmax + 8));
            double* b2 = malloc(sizeof(double) * 2 * (size_t)(mmax + 8));
            if (dir == 0) {
                for (int i = 0; i <= nx; i++)
                    btd[BXIDX(c, i, j)] = multi ? swept_beta_bodies(c, Ls, Le, Ps, Pe, 0, i, j, b1, b2)
                                                : swept_beta(c, Ls, Le, &Ps[0], 0, i, j, b1, b2);
            } else {
                for (int i = 0; i < nx; i++)
                    btd[BYIDX(c, i, j)] = multi ? swept_beta_bodies(c, Ls, Le, Ps, Pe, 1, i, j, b1, b2)
                                                : swept_beta(c, Ls, Le, &Ps[0], 1, i, j, b1, b2);
            }
            free(b1);
            free(b2);
        }
    }

    /* --- 3. per-cell sweep geometry, states and wall quantities --- */
    cellinfo* ci = calloc(nc, sizeof(cellinfo));
    double* Q = malloc(sizeof(double) * 4 * nc);
    unsigned char* has = calloc(nc, 1);
    int bad_body = 0;
    /* each cell's quantities depend on its own inputs only (rows in any order) */
#pragma omp parallel for schedule(static) reduction(| : bad_body)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            size_t k = CIDX(c, i, j);
            cellinfo* e = &ci[k];
            e->as = Ls->alpha[k];
            e->ae = Le->alpha[k];
            e->ab = 0.5 * (e->as + e->ae);
            if (uncov[k] == 1) {
                has[k] = 1;
                for (int m = 0; m < 4; m++) Q[m * nc + k] = Qinit[m * nc + k];
            } else if (uncov[k] == 2) {
                has[k] = 1;
                for (int m = 0; m < 4; m++) Q[m * nc + k] = U1[m * nc + k] / e->ae;
            } else if (e->as > 0.0 && U1[k] > 0.0) { /* live: open volume and content */
                has[k] = 1;
                for (int m = 0; m < 4; m++) Q[m * nc + k] = U1[m * nc + k] / e->as;
            }
            /* time-averaged apertures of the four faces (linear in time, reading R10) */
            double bw, be, bs, bn;
            if (dir == 0) {
                bw = btd[BXIDX(c, i, j)];
                be = btd[BXIDX(c, i + 1, j)];
                bs = beta_avg_y(c, Ls, Le, i, j);
                bn = beta_avg_y(c, Ls, Le, i, j + 1);
            } else {
                bw = beta_avg_x(c, Ls, Le, i, j);
                be = beta_avg_x(c, Ls, Le, i + 1, j);
                bs = btd[BYIDX(c, i, j)];
                bn = btd[BYIDX(c, i, j + 1)];
            }
            /* effective wall vector: integral of the solid-pointing normal over the wall */
            double Nx = (bw - be) * c->hy, Ny = (bs - bn) * c->hx;
            e->wall = e->ab > 0.0 && (Nx != 0.0 || Ny != 0.0);
            if (!e->wall) continue;
            /* unit normal: the time average of the wall's unit normal over the sweep (end of
             * Sec. 2.3.4), the normalised sum of the unit normals of the start and end levels,
             * each from that level's apertures (exact for a planar wall); a level where the
             * cell has no wall adds nothing; without either, the effective vector's direction */
            double sx = 0.0, sy = 0.0;
            for (int lv = 0; lv < 2; lv++) {
                const level_t* L = lv == 0 ? Ls : Le;
                double lx = (beta_x(c, L, i, j) - beta_x(c, L, i + 1, j)) * c->hy;
                double ly = (beta_y(c, L, i, j) - beta_y(c, L, i, j + 1)) * c->hx;
                double ll = sqrt(lx * lx + ly * ly);
                if (ll > 0.0) {
                    sx += lx / ll;
                    sy += ly / ll;
                }
            }
            double nn = sqrt(sx * sx + sy * sy);
            if (nn > 0.0) {
                e->nx = sx / nn;
                e->ny = sy / nn;
            } else {
                nn = sqrt(Nx * Nx + Ny * Ny);
                e->nx = Nx / nn;
                e->ny = Ny / nn;
            }
            /* wall velocity at the mean of the level wall points, at mid-step (R24) */
            double wx, wy;
            int cs = cell_is_cut(c, Ls, i, j), ce = cell_is_cut(c, Le, i, j);
            if (cs && ce) {
                double ax, ay, bx2, by2;
                wall_point(c, Ls, i, j, &ax, &ay);
                wall_point(c, Le, i, j, &bx2, &by2);
                wx = 0.5 * (ax + bx2);
                wy = 0.5 * (ay + by2);
            } else if (cs) {
                wall_point(c, Ls, i, j, &wx, &wy);
            } else {
                wall_point(c, Le, i, j, &wx, &wy);
            }
            /* the body that cuts the cell (several bodies: the one cutting it at level s,
             * else at level e; reading R30) */
            int body = 0;
            if (Ls->cbody) {
                int bs_ = Ls->cbody[k], be_ = Le->cbody[k];
                body = cs && bs_ >= 0 ? bs_ : (be_ >= 0 ? be_ : 0);
                if (cs && ce && bs_ >= 0 && be_ >= 0 && bs_ != be_) bad_body = 1;
            }
            body_velocity(c, body, thalf, wx, wy, &e->uwx, &e->uwy);
            double blo = dir == 0 ? bw : bs, bhi = dir == 0 ? be : bn;
            double mn = blo < bhi ? blo : bhi;
            double sh = fabs(bhi - blo);
            double ah = e->ab - mn;
            if (ah < 0.0) ah = 0.0;
            if (ah > sh) ah = sh;
            e->ahat = ah;
            if (!has[k]) continue; /* emptied cell that found no donors */
            double q[4] = {Q[k], Q[nc + k], Q[2 * nc + k], Q[3 * nc + k]};
            double pst, rst;
            wall_riemann(q, e->nx, e->ny, e->uwx, e->uwy, g, &pst, &rst);
            e->pst = pst;
            /* boundary state Q^B (Sec. 2.3.3): wall normal velocity, the fluid's tangential
             * velocity (the mirror state keeps it), star density and pressure (reading R5) */
            double u = q[1] / q[0], v = q[2] / q[0];
            double un = u * e->nx + v * e->ny, wn = e->uwx * e->nx + e->uwy * e->ny;
            double usx = (u - un * e->nx) + wn * e->nx;
            double usy = (v - un * e->ny) + wn * e->ny;
            e->usx = usx;
            e->usy = usy;
            /* advective part from one common interface state per step: the boundary state
             * of the step's first sweep (Sec. 2.2; reading R8) */
            double qb[4];
            if (first || c->stamp0[k] != c->step) {
                qb[0] = rst;
                qb[1] = rst * usx;
                qb[2] = rst * usy;
                qb[3] = pst / (g - 1.0) + 0.5 * rst * (usx * usx + usy * usy);
                if (first) {
                    for (int m = 0; m < 4; m++) c->Q0[m * nc + k] = qb[m];
                    c->stamp0[k] = c->step;
                }
            } else {
                for (int m = 0; m < 4; m++) qb[m] = c->Q0[m * nc + k];
            }
            for (int m = 0; m < 4; m++) e->qb[m] = qb[m];
            /* F^B = F^ad(Q^B_0) + F^pr(Q^B) in the sweep direction */
            double ua = (dir == 0 ? qb[1] : qb[2]) / qb[0];
            double us = dir == 0 ? usx : usy;
            e->fb[0] = ua * qb[0];
            e->fb[1] = ua * qb[1] + (dir == 0 ? pst : 0.0);
            e->fb[2] = ua * qb[2] + (dir == 1 ? pst : 0.0);
            e->fb[3] = ua * qb[3] + pst * us;
        }

    if (bad_body) c->status |= 4;

    /* --- 4. line-by-line: standard fluxes, stabilised fluxes, update --- */
    double* U2 = malloc(sizeof(double) * 4 * nc);
    int nl = dir == 0 ? ny : nx;  /* number of lines */
    int n = dir == 0 ? nx : ny;   /* cells per line */
    int bclo = dir == 0 ? c->cfg.bc[0] : c->cfg.bc[2];
    int bchi = dir == 0 ? c->cfg.bc[1] : c->cfg.bc[3];
    int nd = 1 + dir;
    /* budget terms per line, added up in line order after the loop (lines are independent
     * and may run in any order) */
    double(*lbnd)[4] = calloc((size_t)nl, sizeof(double[4]));
    double(*lwall)[4] = calloc((size_t)nl, sizeof(double[4]));
#pragma omp parallel for schedule(static)
    for (int line = 0; line < nl; line++) {
        /* per-line buffers with two ghost cells on each side: index p+2 for cell p */
        double(*lq)[4] = malloc(sizeof(double[4]) * (n + 4));
        unsigned char* lh = malloc(n + 4);
        double(*el)[4] = malloc(sizeof(double[4]) * (n + 4));
        double(*er)[4] = malloc(sizeof(double[4]) * (n + 4));
        double(*F)[4] = malloc(sizeof(double[4]) * (n + 1));
        double(*PHI)[4] = malloc(sizeof(double[4]) * (n + 1));
        double* bt = malloc(sizeof(double) * (n + 1));
#define CELL(p) (dir == 0 ? CIDX(c, (p), line) : CIDX(c, line, (p)))
        for (int p = 0; p < n; p++) {
            size_t k = CELL(p);
            lh[p + 2] = has[k];
            for (int m = 0; m < 4; m++) lq[p + 2][m] = has[k] ? Q[m * nc + k] : 0.0;
        }
        /* ghost cells: zero-gradient copy, or mirror with negated normal momentum */
        for (int gph = 0; gph < 2; gph++) {
            int src_lo = gph, dst_lo = 1 - gph;      /* ghost -1 <- cell 0, ghost -2 <- cell 1 or 0 */
            int src_hi = n - 1 - gph, dst_hi = n + 2 + gph;
            int slo = bclo == 1 ? src_lo : 0;
            int shi = bchi == 1 ? src_hi : n - 1;
            if (slo >= n) slo = n - 1;
            if (shi < 0) shi = 0;
            lh[dst_lo] = lh[slo + 2];
            lh[dst_hi] = lh[shi + 2];
            for (int m = 0; m < 4; m++) {
                lq[dst_lo][m] = lq[slo + 2][m];
                lq[dst_hi][m] = lq[shi + 2][m];
            }
            if (bclo == 1) lq[dst_lo][nd] = -lq[dst_lo][nd];
            if (bchi == 1) lq[dst_hi][nd] = -lq[dst_hi][nd];
        }
        /* face apertures along the line */
        for (int f = 0; f <= n; f++)
            bt[f] = dir == 0 ? btd[BXIDX(c, f, line)] : btd[BYIDX(c, line, f)];
        /* reconstruction + half-step evolution for cells -1 .. n (ghosts included) */
        for (int p = -1; p <= n; p++) {
            int x = p + 2;
            if (!lh[x]) continue;
            int ok = lh[x - 1] && lh[x + 1];
            muscl_cell(lq[x - 1], lq[x], lq[x + 1], ok, lam, dir, g, el[x], er[x]);
        }
        /* standard fluxes on faces with an open aperture and states on both sides */
        for (int f = 0; f <= n; f++) {
            int xl = f + 1, xr = f + 2; /* cells f-1 and f */
            int act = bt[f] > 0.0 && lh[xl] && lh[xr];
            if (!act) {
                for (int m = 0; m < 4; m++) F[f][m] = 0.0, PHI[f][m] = 0.0;
                continue;
            }
            hllc(er[xl], el[xr], dir, g, F[f]);
            /* stabilised, aperture-weighted flux in division-free form:
             * beta F2D = beta F - (s_L - ahat_L)(F - FB_L) - (s_R - ahat_R)(F - FB_R)
             * (Eqs. Klein2shieldedFluxMethod2 and Klein2DtotalfluxaMethod2, with the shielded
             * flux of the same face, reading R1/R2) */
            const cellinfo* L = f > 0 ? &ci[CELL(f - 1)] : NULL;
            const cellinfo* R = f < n ? &ci[CELL(f)] : NULL;
            double sL = 0.0, sR = 0.0;
            if (L && L->wall) {
                double d = bt[f] - bt[f - 1];
                sL = d > 0.0 ? d : 0.0;
            }
            if (R && R->wall) {
                double d = bt[f] - bt[f + 1];
                sR = d > 0.0 ? d : 0.0;
            }
            double kap = 1.0;
            if (sL + sR > bt[f]) kap = bt[f] / (sL + sR);
            double cL = sL > 0.0 ? kap * (sL - L->ahat) : 0.0;
            double cR = sR > 0.0 ? kap * (sR - R->ahat) : 0.0;
            for (int m = 0; m < 4; m++) {
                double phi = bt[f] * F[f][m];
                if (cL != 0.0) phi = phi - cL * (F[f][m] - L->fb[m]);
                if (cR != 0.0) phi = phi - cR * (F[f][m] - R->fb[m]);
                PHI[f][m] = phi;
            }
        }
        /* conservative update (Eqs. Klein2DcompleteMovingMethod2a/b): the wall contributes
         * only its pressure term (Eq. Klein2DMovingResultantFluxes, readings R3-R5) */
        for (int p = 0; p < n; p++) {
            size_t k = CELL(p);
            const cellinfo* e = &ci[k];
            if (!has[k]) {
                for (int m = 0; m < 4; m++) U2[m * nc + k] = 0.0;
                continue;
            }
            double W[4] = {0, 0, 0, 0};
            if (e->wall) {
                /* wall term of Eqs. Klein2DcompleteMovingMethod2a/b: dbeta (F^B - u_wall^d Q^B),
                 * dbeta = beta_hi - beta_lo (readings R3, R4) */
                double db = bt[p + 1] - bt[p];
                double ud = dir == 0 ? e->uwx : e->uwy;
                for (int m = 0; m < 4; m++) W[m] = db * (e->fb[m] - ud * e->qb[m]);
                for (int m = 0; m < 4; m++) lwall[line][m] += lam * W[m] * area;
            }
            for (int m = 0; m < 4; m++)
                U2[m * nc + k] = U1[m * nc + k] + lam * ((PHI[p][m] - PHI[p + 1][m]) + W[m]);
            if ((dir == 0 ? p : line) == c->trace_i && (dir == 0 ? line : p) == c->trace_j) {
                double* r = c->trace;
                for (int m = 0; m < 4; m++) {
                    r[m] = F[p][m];
                    r[4 + m] = F[p + 1][m];
                    r[8 + m] = PHI[p][m];
                    r[12 + m] = PHI[p + 1][m];
                    r[16 + m] = e->wall ? e->fb[m] : 0.0;
                    r[20 + m] = Q[m * nc + k];
                }
                r[24] = e->as;
                r[25] = e->ae;
                r[26] = bt[p];
                r[27] = bt[p + 1];
                r[28] = e->ahat;
                r[29] = e->wall;
                r[30] = has[k];
            }
        }
        for (int m = 0; m < 4; m++) lbnd[line][m] = lam * (PHI[0][m] - PHI[n][m]) * area;
#undef CELL
        free(lq);
        free(lh);
        free(el);
        free(er);
        free(F);
        free(PHI);
        free(bt);
    }
    for (int line = 0; line < nl; line++)
        for (int m = 0; m < 4; m++) {
            c->bnd[m] += lbnd[line][m];
            c->wall[m] += lwall[line][m];
        }
    free(lbnd);
    free(lwall);

    /* --- 5. collapse: a live cell whose updated content is not an admissible gas state
     *        (rho <= 0 or p <= 0) is emptied like a covered cell and refilled at the start
     *        of the next sweep like an uncovered cell (reading R27) --- */
    unsigned char* gone = calloc(nc, 1);
    for (size_t k = 0; k < nc; k++) {
        if (ci[k].as > 0.0 && ci[k].ae == 0.0) {
            gone[k] = 1; /* covered */
        } else if (ci[k].ae > 0.0 && has[k]) {
            double r = U2[k], e = U2[3 * nc + k];
            double mx = U2[nc + k], my = U2[2 * nc + k];
            if (!(r > 0.0) || !(e - 0.5 * (mx * mx + my * my) / r > 0.0)) gone[k] = 2;
        }
    }

    /* --- 6. covering (Eqs. massDeficitEquation, cutCellCoverDonation): residual of cells
     *        that became solid (or collapsed), shared by their neighbours by volume
     *        (reading R14) --- */
    double* U3 = malloc(sizeof(double) * 4 * nc);
    memcpy(U3, U2, sizeof(double) * 4 * nc);
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            size_t k = CIDX(c, i, j);
            if (!gone[k]) continue;
            int rec[8], nr = 0;
            for (int pass = 0; pass < 2 && nr == 0; pass++) {
                int cnt = pass == 0 ? 4 : 8;
                for (int q = 0; q < cnt; q++) {
                    int ii = i + d8[q][0], jj = j + d8[q][1];
                    if (ii < 0 || ii >= nx || jj < 0 || jj >= ny) continue;
                    size_t kk = CIDX(c, ii, jj);
                    if (Le->alpha[kk] > 0.0 && !gone[kk]) rec[nr++] = (int)kk;
                }
            }
            if (nr == 0) {
                for (int m = 0; m < 4; m++) c->lost[m] += U2[m * nc + k] * area;
            } else {
                double den = 0.0;
                for (int q = 0; q < nr; q++) den += Le->alpha[rec[q]];
                for (int q = 0; q < nr; q++) {
                    double w = Le->alpha[rec[q]] / den;
                    for (int m = 0; m < 4; m++) U3[m * nc + rec[q]] += w * U2[m * nc + k];
                }
            }
            for (int m = 0; m < 4; m++) U3[m * nc + k] = 0.0;
        }

    /* --- 7. collapse after covering (reading R28): a cell left with content that is not an
     *        admissible gas state once the residuals have been added is emptied in the same
     *        way, its content going to its face neighbours that stay fluid, are not emptied
     *        and are admissible (else its eight neighbours), weighted by alpha_e.  All cells
     *        of a round move their content at once; two rounds, and a cell still inadmissible
     *        after them is reported (status bit 2). --- */
    for (int round = 0; round < 2; round++) {
        unsigned char* bad = calloc(nc, 1);
        int nbad = 0;
        for (size_t k = 0; k < nc; k++) {
            if (!(Le->alpha[k] > 0.0) || gone[k]) continue;
            double r = U3[k], mx = U3[nc + k], my = U3[2 * nc + k], e = U3[3 * nc + k];
            if (r == 0.0 && mx == 0.0 && my == 0.0 && e == 0.0) continue; /* no content */
            if (!(r > 0.0) || !(e - 0.5 * (mx * mx + my * my) / r > 0.0)) {
                bad[k] = 1;
                nbad++;
            }
        }
        if (nbad == 0) {
            free(bad);
            break;
        }
        double* U4 = malloc(sizeof(double) * 4 * nc);
        memcpy(U4, U3, sizeof(double) * 4 * nc);
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t k = CIDX(c, i, j);
                if (!bad[k]) continue;
                int rec[8], nr = 0;
                for (int pass = 0; pass < 2 && nr == 0; pass++) {
                    int cnt = pass == 0 ? 4 : 8;
                    for (int q = 0; q < cnt; q++) {
                        int ii = i + d8[q][0], jj = j + d8[q][1];
                        if (ii < 0 || ii >= nx || jj < 0 || jj >= ny) continue;
                        size_t kk = CIDX(c, ii, jj);
                        if (Le->alpha[kk] > 0.0 && !gone[kk] && !bad[kk]) rec[nr++] = (int)kk;
                    }
                }
                if (nr == 0) {
                    for (int m = 0; m < 4; m++) c->lost[m] += U3[m * nc + k] * area;
                } else {
                    double den = 0.0;
                    for (int q = 0; q < nr; q++) den += Le->alpha[rec[q]];
                    for (int q = 0; q < nr; q++) {
                        double w = Le->alpha[rec[q]] / den;
                        for (int m = 0; m < 4; m++) U4[m * nc + rec[q]] += w * U3[m * nc + k];
                    }
                }
                for (int m = 0; m < 4; m++) U4[m * nc + k] = 0.0;
                gone[k] = 2;
            }
        memcpy(U3, U4, sizeof(double) * 4 * nc);
        free(U4);
        free(bad);
    }
    for (size_t k = 0; k < nc; k++) {
        if (!(Le->alpha[k] > 0.0) || gone[k]) continue;
        double r = U3[k], mx = U3[nc + k], my = U3[2 * nc + k], e = U3[3 * nc + k];
        if (r == 0.0 && mx == 0.0 && my == 0.0 && e == 0.0) continue;
        if (!(r > 0.0) || !(e - 0.5 * (mx * mx + my * my) / r > 0.0)) c->status |= 2;
    }
    memcpy(c->U, U3, sizeof(double) * 4 * nc);
    free(btd);
    free(Qinit);
    free(uncov);
    for (size_t k = 0; k < nc; k++) c->ncollapse += gone[k] == 2;
    free(gone);
    free(U1);
    free(U2);
    free(U3);
    free(Q);
    free(has);
    free(ci);
    c->sweeps_done++;
    return 0;
}

/* Start a split step of size dt: pose the body at t^{n+1}, build the stage level (first
 * sweep's direction moves the polygon, the other coordinate stays; reading R11) and the
 * end level. */
/* Axisymmetric form (option bit 0; reading R33; the shock tube of Sec. 3.5 uses the Euler
 * equations in axisymmetric form): in (x, r) with r = y the equations carry the geometric
 * source S = -(1/r) (rho v, rho u v, rho v^2, v (E + p)).  It is applied as an operator step
 * of length dt before the split step's first sweep, to the content per cell volume (S is
 * homogeneous of degree one in the state, so S(U) = alpha S(Q), p from U as from Q), with r
 * the radius of the cell centre; cells without content are skipped. */
static void axisym_source(ccref_ctx* c, double dt) {
    size_t nc = (size_t)c->cfg.nx * c->cfg.ny;
    double g = c->cfg.gamma;
    for (int j = 0; j < c->cfg.ny; j++) {
        double r = vy_of(c, j) + 0.5 * c->hy;
        double f = dt / r;
        for (int i = 0; i < c->cfg.nx; i++) {
            size_t k = CIDX(c, i, j);
            double rho = c->U[k], mx = c->U[nc + k], my = c->U[2 * nc + k], e = c->U[3 * nc + k];
            if (!(rho > 0.0)) continue;
            double v = my / rho;
            double p = (g - 1.0) * (e - 0.5 * (mx * mx + my * my) / rho);
            c->U[k] = rho - f * my;
            c->U[nc + k] = mx - f * (mx * v);
            c->U[2 * nc + k] = my - f * (my * v);
            c->U[3 * nc + k] = e - f * (v * (e + p));
        }
    }
}

int ccref_begin_step(ccref_ctx* c, double dt) {
    if (c->in_step || !(dt > 0.0)) return 1;
    if (c->cfg.options & 1) axisym_source(c, dt);
    double t1 = c->t + dt;
    if (c->parity == 0)
        level_posed(c, t1, c->t, &c->L[c->sm]);
    else
        level_posed(c, c->t, t1, &c->L[c->sm]);
    level_at_time(c, t1, &c->L[c->s1]);
    for (int b = 0; b < c->nb; b++) {
        body_t* B = &c->B[b];
        double th0 = B->theta0 + B->amp * sin(B->omega * c->t);
        double th1 = B->theta0 + B->amp * sin(B->omega * t1);
        B->cosd = cos(th1 - th0);
        B->sind = sin(th1 - th0);
        B->c0x = B->ref_x + B->vx * c->t;
        B->c0y = B->ref_y + B->vy * c->t;
        B->c1x = B->ref_x + B->vx * t1;
        B->c1y = B->ref_y + B->vy * t1;
    }
    c->in_step = 1;
    c->sweeps_done = 0;
    c->step_dt = dt;
    return 0;
}

int ccref_end_step(ccref_ctx* c) {
    if (!c->in_step || c->sweeps_done != 2) return 1;
    int old = c->s0;
    c->s0 = c->s1;
    c->s1 = old;
    c->t = c->t + c->step_dt;
    c->step++;
    c->parity ^= 1;
    c->in_step = 0;
    return 0;
}

/* One full split step: x then y on even steps, y then x on odd steps (Sec. 2.3.4 end). */
int ccref_step(ccref_ctx* c, double dt) {
    if (ccref_begin_step(c, dt)) return 1;
    int d1 = c->parity, d2 = 1 - c->parity;
    if (ccref_sweep(c, d1, dt)) return 1;
    if (ccref_sweep(c, d2, dt)) return 1;
    return ccref_end_step(c);
}

/* ------------------------------------------------------------------------------------ */
/* Pure building blocks exported for unit tests.                                        */
/* ------------------------------------------------------------------------------------ */
void ccref_hllc(const double* ql, const double* qr, int d, double g, double* f) { hllc(ql, qr, d, g, f); }
void ccref_flux(const double* q, int d, double g, double* f) { euler_flux(q, d, g, f); }
double ccref_vanleer(double a, double b) { return vanleer(a, b); }
void ccref_muscl(const double* qm, const double* q, const double* qp, int ok, double lam, int d,
                 double g, double* el, double* er) {
    muscl_cell(qm, q, qp, ok, lam, d, g, el, er);
}
void ccref_wall_riemann(const double* q, double nx, double ny, double wx, double wy, double g,
                        double* out2) {
    wall_riemann(q, nx, ny, wx, wy, g, out2, out2 + 1);
}
/* Rigid-body velocity of the body point at (x, y) at time t (out2: ux, uy). */
void ccref_body_velocity(const ccref_ctx* c, double t, double x, double y, double* out2) {
    body_velocity(c, 0, t, x, y, out2, out2 + 1);
}
/* Displacement along d of the point (x, y) under the rigid map of the open step. */
double ccref_step_disp(const ccref_ctx* c, int d, double x, double y) {
    return c->in_step ? step_disp(c, 0, d, x, y) : NAN;
}
/* Record the sweep quantities of cell (i, j) in every later sweep (i < 0: stop). */
int ccref_trace(ccref_ctx* c, int i, int j) {
    c->trace_i = i;
    c->trace_j = j;
    for (int k = 0; k < TRACE_N; k++) c->trace[k] = NAN;
    return 0;
}
int ccref_trace_get(const ccref_ctx* c, double* out) {
    for (int k = 0; k < TRACE_N; k++) out[k] = c->trace[k];
    return TRACE_N;
}
/* Oracle-only options.  1: a cell that becomes fluid takes content from its donors as
 * printed (Eqs. cutCellInitialisation, cutCellInitialisationDonorCellUpdate) instead of a
 * state only (reading R13); kept to show why R13 is used. */
int ccref_set_option(ccref_ctx* c, int opt, int value) {
    if (opt != 1) return 1;
    c->uncover_moves_content = value != 0;
    return 0;
}
/* Area of the posed polygon clipped to a rectangle (for tests). */
double ccref_clip_area(const double* poly, int m, double ox, double oy, double w, double h) {
    double* b1 = malloc(sizeof(double) * 2 * (size_t)(m + 8));
    double* b2 = malloc(sizeof(double) * 2 * (size_t)(m + 8));
    double a = clip_area(poly, m, ox, oy, w, h, b1, b2);
    free(b1);
    free(b2);
    return a;
}

/* Wall pressure distribution at level n (the surface pressure of the pitching aerofoil,
 * Sec. 3.6): for every cell with fluid content and a non-zero effective wall normal, in
 * increasing linear index j nx + i, six values: the index, the wall point (x, y), p* of the
 * wall Riemann problem and the normal N (Nx, Ny) -- the terms ccref_surface_loads sums.
 * Writes at most max records to out (6 max doubles); returns the number of records. */
int ccref_surface_pressure(const ccref_ctx* c, double* out, int max) {
    if (c->nb == 1 && c->B[0].m == 0) return 0;
    const level_t* L = &c->L[c->s0];
    size_t nc = (size_t)c->cfg.nx * c->cfg.ny;
    int n = 0;
    for (int j = 0; j < c->cfg.ny; j++)
        for (int i = 0; i < c->cfg.nx; i++) {
            size_t k = CIDX(c, i, j);
            double a = L->alpha[k];
            if (!(a > 0.0) || !(c->U[k] > 0.0)) continue;
            double Nx = (beta_x(c, L, i, j) - beta_x(c, L, i + 1, j)) * c->hy;
            double Ny = (beta_y(c, L, i, j) - beta_y(c, L, i, j + 1)) * c->hx;
            if (Nx == 0.0 && Ny == 0.0) continue;
            double q[4];
            for (int m = 0; m < 4; m++) q[m] = c->U[m * nc + k] / a;
            double nn = sqrt(Nx * Nx + Ny * Ny);
            double wx, wy, uwx, uwy, ps, rs;
            wall_point(c, L, i, j, &wx, &wy);
            body_velocity(c, L->cbody ? L->cbody[k] : 0, c->t, wx, wy, &uwx, &uwy);
            wall_riemann(q, Nx / nn, Ny / nn, uwx, uwy, c->cfg.gamma, &ps, &rs);
            if (n < max) {
                double* r = out + 6 * (size_t)n;
                r[0] = (double)k;
                r[1] = wx;
                r[2] = wy;
                r[3] = ps;
                r[4] = Nx;
                r[5] = Ny;
            }
            n++;
        }
    return n;
}

/* Surface loads at level n (post-processing of the pitching aerofoil of Sec. 3.6; reading:
 * the sum over the cells with fluid content of p* N, p* the wall pressure of the wall
 * Riemann problem (Eq. riemann_wallvel, reading R9) between the cell state U/alpha and its
 * mirror image moving with the body at the cell's wall point, N the level's effective wall
 * normal ((beta_W - beta_E) hy, (beta_S - beta_N) hx), pointing into the body, reading
 * R12).  out4: Fx, Fy, the moment about the body's pose origin, and sum p* |N|.  Plain
 * sums in row-major cell order.  With several bodies: the loads on body b (the wall cells
 * the body cuts at level n). */
int ccref_surface_loads_body(const ccref_ctx* c, int b, double* out4) {
    for (int k = 0; k < 4; k++) out4[k] = 0.0;
    if (b < 0 || b >= c->nb) return 1;
    if (c->B[b].m == 0) return 0;
    const level_t* L = &c->L[c->s0];
    size_t nc = (size_t)c->cfg.nx * c->cfg.ny;
    const body_t* B = &c->B[b];
    double cx = B->ref_x + B->vx * c->t, cy = B->ref_y + B->vy * c->t;
    for (int j = 0; j < c->cfg.ny; j++)
        for (int i = 0; i < c->cfg.nx; i++) {
            size_t k = CIDX(c, i, j);
            double a = L->alpha[k];
            if (!(a > 0.0) || !(c->U[k] > 0.0)) continue;
            if (L->cbody && L->cbody[k] != b) continue;
            double Nx = (beta_x(c, L, i, j) - beta_x(c, L, i + 1, j)) * c->hy;
            double Ny = (beta_y(c, L, i, j) - beta_y(c, L, i, j + 1)) * c->hx;
            if (Nx == 0.0 && Ny == 0.0) continue;
            double q[4];
            for (int m = 0; m < 4; m++) q[m] = c->U[m * nc + k] / a;
            double nn = sqrt(Nx * Nx + Ny * Ny);
            double wx, wy, uwx, uwy, ps, rs;
            wall_point(c, L, i, j, &wx, &wy);
            body_velocity(c, b, c->t, wx, wy, &uwx, &uwy);
            wall_riemann(q, Nx / nn, Ny / nn, uwx, uwy, c->cfg.gamma, &ps, &rs);
            out4[0] += ps * Nx;
            out4[1] += ps * Ny;
            out4[2] += (wx - cx) * (ps * Ny) - (wy - cy) * (ps * Nx);
            out4[3] += ps * nn;
        }
    return 0;
}

int ccref_surface_loads(const ccref_ctx* c, double* out4) { return ccref_surface_loads_body(c, 0, out4); }

int ccref_nbodies(const ccref_ctx* c) { return c->nb; }

/* Body of each cut cell of a level with several bodies (-1 elsewhere); returns 1 for a
 * context with one body. */
int ccref_cell_bodies(const ccref_ctx* c, int which, int8_t* out) {
    int s = slot_of(c, which);
    if (s < 0 || !c->L[s].cbody) return 1;
    memcpy(out, c->L[s].cbody, (size_t)c->cfg.nx * c->cfg.ny);
    return 0;
}
