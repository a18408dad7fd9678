// Host side of the cut-cell library: contexts, batches, workspace carving, body posing,
// level bookkeeping, per-step argument blocks and the launch sequence of the split step.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/cc.h"
#include "cc_device.h"
#include "engine.h"
#include "persist.h"
#include "plan.h"
#include "loads.h"
#include "geometry.h"
#include "reduce.h"
#include "sweep.h"
#include "lists.h"

using namespace cc;

namespace {

constexpr size_t ALIGN = 256;
constexpr int NPART = 1024;  // blocks of the deterministic sum
constexpr int TPB = 256;
constexpr int CFL_MAX_BLOCKS = 512;

size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Dense-sweep tile variants: rows per block of the x-sweep, rows per tile of the y-sweep
// (the y tile lives in LDS: (2 TR + 7) x 64 x 4 values, kept within 64 KiB).
// y-sweep variants 0-3: 64-column tiles staged in LDS; 4-5: column walks of 256 columns
constexpr int NX_VARIANTS = 4, NY_VARIANTS = 6;
constexpr int X_RB[NX_VARIANTS] = {1, 2, 4, 8};
constexpr int Y_TR[NY_VARIANTS] = {8, 12, 16, 24, 4, 8};
constexpr bool y_walk(int v) { return v >= 4; }

bool dense_variant_ok(int prec, int dir, int v) {
    size_t rs = prec == CC_FP32_GEOM64 ? 4 : 8;
    if (dir == 0) return v >= 0 && v < NX_VARIANTS;
    if (v < 0 || v >= NY_VARIANTS) return false;
    if (y_walk(v)) return rs == 4 || Y_TR[v] <= 4;  // an FP64 walk of 8 rows spills registers
    return (size_t)(2 * Y_TR[v] + 7) * 64 * 4 * rs <= 65536;
}
int dense_blocks(int dir, int v, int nx, int ny) {
    if (dir == 0) {
        int rb = X_RB[v];
        return ((nx + DX_OUT - 1) / DX_OUT) * ((ny + rb - 1) / rb);
    }
    int tr = Y_TR[v];
    if (y_walk(v)) return ((nx + DYC_T - 1) / DYC_T) * ((ny + tr - 1) / tr);
    return ((nx + 63) / 64) * ((ny + tr - 1) / tr);
}

// --------------------------------------------------------------------------- workspace
constexpr int DTLOG = 1024;  // steps of one device-planned run between read-backs

struct Layout {
    size_t nc, nvx, nfx, nfy, cap, capf;
    size_t u_bytes;
    size_t off_u[2], off_vcls[3], off_fx[3], off_fy[3], off_alpha[3], off_poly[3];
    size_t off_body;
    size_t off_qb, off_stamp;
    size_t off_sQ, off_sU1, off_shas, off_sbt[2], off_swall, off_sfb, off_swv, off_sahat, off_sU2, off_sgone;
    size_t off_sf1, off_sf2, off_nbad;
    size_t off_sync;
    size_t off_args, off_offs, off_cflout;
    size_t off_smax, off_status, off_ncol, off_part, off_tot, off_spd;
    size_t off_pconst, off_pstate, off_dtlog;
    size_t off_budget, off_bslot;
    size_t off_cbody[3];     // several bodies: the body of each cut cell, per level slot
    size_t set_bytes;        // several bodies: the bodies' block after the argument block
    int bs_patch, bs_cover;  // offsets (doubles) of the patch and covering budget slots
    size_t total;
    int capw, caph;  // sweep-box capacity (cells)
    int spd_dense;   // speed slot pairs the dense tiles share (NSPD)
    int gw, gh;      // geometry-region capacity (cells)
};

int body_m(const cc_body* b) { return b && b->nverts > 0 && b->verts ? b->nverts : 0; }

// Several bodies: per level slot their posed polygons, per body the step's motion, then the
// posed vertices (slot s, body b at vertex s * mtot + first vertex of b), uploaded with the
// argument block of every step.
struct BodySet {
    Poly poly[3][MAX_BODIES];
    Motion mot[MAX_BODIES];
};
constexpr size_t SET_VERTS = (sizeof(BodySet) + 15) / 16 * 16;
size_t bodyset_bytes(int mtot) { return SET_VERTS + 3 * 16 * (size_t)mtot; }
constexpr int BODY_MAX_VERTS = 256;  // vertices of each of several bodies

// True for a polygon of at least three finite vertices whose every turn is to the left
// (or straight on), with a positive signed area and one full turn in total (a polygon
// that winds round twice turns left everywhere too); repeated vertices are allowed.  The
// geometry's chain searches assume a convex polygon in counter-clockwise order.
bool convex_ccw(const double* v, int m) {
    if (m < 3) return false;
    std::vector<double> ex, ey;  // the edges of nonzero length, in order
    double area2 = 0.0;
    for (int k = 0; k < m; k++) {
        int k1 = (k + 1) % m;
        double ax = v[2 * k], ay = v[2 * k + 1], bx = v[2 * k1], by = v[2 * k1 + 1];
        if (!std::isfinite(ax) || !std::isfinite(ay)) return false;
        if (bx != ax || by != ay) {
            ex.push_back(bx - ax);
            ey.push_back(by - ay);
        }
        area2 += ax * by - bx * ay;
    }
    size_t n = ex.size();
    if (n < 3 || !(area2 > 0.0)) return false;
    double turn = 0.0;
    for (size_t k = 0; k < n; k++) {
        size_t k1 = (k + 1) % n;
        double cr = ex[k] * ey[k1] - ey[k] * ex[k1];
        if (cr < 0.0) return false;
        turn += std::atan2(cr, ex[k] * ex[k1] + ey[k] * ey[k1]);
    }
    return std::fabs(turn - 2.0 * M_PI) < 1e-6;
}

// nbodies >= 2: b points to that many bodies; their geometry and box phases cover the whole
// grid (the bodies' boxes may span it, and their union moves with their relative motion).
Layout make_layout(const cc_config* c, const cc_body* b, int nbodies = 1) {
    Layout L{};
    size_t nx = c->nx, ny = c->ny;
    bool multi = nbodies > 1;
    int m = multi ? 0 : body_m(b);
    int mtot = 0;
    for (int k = 0; multi && k < nbodies; k++) mtot += b[k].nverts;
    bool hasb = m > 0 || multi;
    L.nc = nx * ny;
    L.nvx = (nx + 1) * (ny + 1);
    L.nfx = ny * (nx + 1);
    L.nfy = (ny + 1) * nx;
    size_t rs = c->precision == CC_FP32_GEOM64 ? sizeof(float) : sizeof(double);
    L.u_bytes = 4 * L.nc * rs;
    // capacities: the body stays inside a disc of radius R about its moving origin
    double R = 0.0;
    for (int k = 0; k < m; k++) R = std::max(R, std::hypot(b->verts[2 * k], b->verts[2 * k + 1]));
    double hx = (c->x_hi - c->x_lo) / c->nx, hy = (c->y_hi - c->y_lo) / c->ny;
    if (multi) {
        L.capw = L.gw = (int)nx;
        L.caph = L.gh = (int)ny;
    } else if (m > 0) {
        double cw = std::ceil(2.0 * R / hx) + 16.0, ch = std::ceil(2.0 * R / hy) + 16.0;
        L.capw = (int)std::min<double>(cw, (double)nx);
        L.caph = (int)std::min<double>(ch, (double)ny);
        L.gw = (int)std::min<double>(cw + 4.0, (double)nx);
        L.gh = (int)std::min<double>(ch + 4.0, (double)ny);
    } else {
        L.capw = L.caph = L.gw = L.gh = 0;
    }
    L.cap = (size_t)L.capw * L.caph;
    L.capf = hasb ? (size_t)(L.capw + 1) * (L.caph + 1) : 0;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += up(std::max<size_t>(bytes, 1));
        return r;
    };
    L.off_u[0] = take(L.u_bytes);
    L.off_u[1] = take(L.u_bytes);
    for (int s = 0; s < 3; s++) {
        L.off_vcls[s] = take(L.nvx);
        L.off_fx[s] = take(L.nfx * 16);
        L.off_fy[s] = take(L.nfy * 16);
        L.off_alpha[s] = take(L.nc * 8);
        L.off_poly[s] = take((size_t)std::max(m, 1) * 16);
    }
    L.off_body = take((size_t)std::max(m, 1) * 16);
    L.off_qb = take(hasb ? 4 * L.nc * 8 : 8);
    L.off_stamp = take(hasb ? L.nc * 4 : 4);
    for (int s = 0; s < 3; s++) L.off_cbody[s] = take(multi ? L.nc : 1);
    size_t cap = std::max<size_t>(L.cap, 1), capf = std::max<size_t>(L.capf, 1);
    L.off_sQ = take(4 * cap * 8);
    L.off_sU1 = take(4 * cap * 8);
    L.off_shas = take(cap);
    L.off_sbt[0] = take(capf * 8);
    L.off_sbt[1] = take(capf * 8);
    L.off_swall = take(cap);
    L.off_sfb = take(4 * cap * 8);
    L.off_swv = take(4 * cap * 8);
    L.off_sahat = take(cap * 8);
    L.off_sU2 = take(4 * cap * 8);
    L.off_sgone = take(cap);
    L.off_sf1 = take(cap);
    L.off_sf2 = take(cap);
    L.off_nbad = take(8);
    L.off_sync = take(sizeof(GridSync));
    L.set_bytes = multi ? bodyset_bytes(mtot) : 0;
    L.off_args = take(sizeof(StepArgs) + L.set_bytes);
    L.off_offs = take((size_t)NKINDS * 3 * 4);
    L.off_cflout = take(24);  // read-back: 2 speed maxima, then status and collapse count
    L.off_smax = take(16);
    L.off_status = take(4);
    L.off_ncol = take(4);
    L.off_part = take(std::max<size_t>(4 * NPART * 8, 2 * CFL_MAX_BLOCKS * 8));
    L.off_tot = take(4 * 8);
    L.spd_dense = NSPD;
    L.off_spd = take((size_t)2 * 8 * ((size_t)L.spd_dense + (std::max<size_t>(L.cap, 1) + T_BOX - 1) / T_BOX));
    L.off_pconst = take(sizeof(PlanConst));
    L.off_pstate = take(sizeof(PlanState));
    L.off_dtlog = take((size_t)DTLOG * 8);
    // budget: running sums, and the per-sweep slots (dense: two per line of either sweep;
    // patch line segments and column tiles: 12 doubles each; covering blocks: 4 each)
    L.off_budget = take(16 * 8);
    size_t dense_slots = 2 * std::max(nx, ny);
    size_t patch_blocks = hasb ? (size_t)std::max(patch_line_blocks<0>(L.capw, L.caph), patch_tile_blocks(L.capw, L.caph)) : 1;
    size_t cover_blocks = (std::max<size_t>(L.cap, 1) + T_BOX - 1) / T_BOX;
    L.bs_patch = (int)(BS_DENSE + 4 * dense_slots);
    L.bs_cover = (int)(L.bs_patch + 12 * patch_blocks);
    L.off_bslot = take(8 * ((size_t)L.bs_cover + 4 * cover_blocks));
    L.total = o;
    return L;
}

struct TimedPair {
    hipEvent_t a, b;
    int kind;
};

// --------------------------------------------------------------------------- engine
// Launch plan for the members of a batch (one member for a context's own calls): per-step
// argument blocks (two pinned host buffers, one device array), per-launch offset tables and
// the captured graphs of a whole step.
struct Engine {
    int prec = CC_FP64;
    int cap_n = 0;
    std::vector<cc_ctx*> mem;
    StepArgs* h_args[2] = {nullptr, nullptr};
    StepArgs* d_args = nullptr;
    int* d_off = nullptr;  // NKINDS tables of (units + 1) entries, stride 2 cap_n + 1
    std::vector<int> h_off[NKINDS];
    // one read-back region of 24 cap_n bytes: 2 speed maxima per member slot, then the
    // status word and collapse count per member
    unsigned long long* d_cflout = nullptr;
    unsigned long long* h_cflout = nullptr;  // pinned
    unsigned int* d_gather = nullptr;        // = d_cflout + 2 cap_n
    unsigned int* h_gather = nullptr;        // = h_cflout + 2 cap_n
    hipEvent_t ev[2] = {nullptr, nullptr};   // last use of host buffer b
    bool ev_used[2] = {false, false};
    int buf = 0;
    int tile_x = 0, tile_y = 1;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int gkey[2] = {-1, -1};
    hipGraphExec_t pexec[3] = {nullptr, nullptr, nullptr};  // device-planned step, by first direction + 1
    hipGraphExec_t pexec_run[3] = {nullptr, nullptr, nullptr};  // PLANNED_RUN such steps, the same way
    int mode = 0;                       // 0: one launch per phase; 1: one persistent launch per sweep
    GridSync* d_sync = nullptr;         // barrier counters of the persistent sweep launches
    unsigned long long wait_ticks = 0;  // barrier wait limit (wall-clock ticks)
    // timing (cc_timing, cc_batch_timing): bit 0 a whole step's launches one by one, the
    // dense (merged wall + dense) launches bracketed by events of their own; bit 1 events
    // around the box and geometry phases of single sweeps.  Event pairs recorded and not
    // read yet, and spare ones.
    int timing = 0;
    std::vector<TimedPair> pending, pool;
    // the box cells' first phase runs in the leading blocks of the sweep's y launch when
    // there is one, else of its x launch when merge_x, else as a launch of its own before
    // the dense launches (see engine_plan)
    bool merge_x = true;
    // a context with several bodies (its own engine only): the box phase's first launch is
    // the several-body kernel, and `extra` bytes of the bodies' block follow the argument
    // block in the host buffers and the upload
    bool multi = false;
    size_t extra = 0;
    // an instance in axisymmetric form (its own engine only): the source launch before the
    // first sweep, over axi_blocks blocks
    bool axisym = false;
    int axi_blocks = 0;
};

// One of several bodies (host copy of its cc_body).
struct HostBody {
    std::vector<double> verts;
    double ref_x, ref_y, theta0, vx, vy, amp, omega;
};

}  // namespace

struct cc_ctx {
    cc_config cfg;
    Grid g;
    hipStream_t stream;
    Layout lay;
    char* ws;
    int m;
    std::vector<double> bverts;
    double ref_x, ref_y, theta0, vx, vy, amp, omega;
    Cert cert0;      // discs of the body turned by theta0 (used while it does not turn)
    Extremes ext0;   // its extreme coordinates and the vertices attaining them
    int cur;  // U[cur] holds the level-n state
    Level lev[3];
    Box lbox[3];  // region of each slot that may differ from all-fluid
    int s0, sm, s1;
    double t;
    int64_t step;
    int parity;
    bool in_step, have_state;
    int sweeps_done;
    double step_dt;
    Motion mot;
    double hx, hy;
    Box last_sweep_box;
    Engine eng;  // launch plan of this context's own calls
    cc_batch* batch;  // batch this context belongs to, if any
    // wave speeds of the current state, reduced and read back by the last captured step
    bool speeds_ready;
    int speeds_buf;
    int advanced;  // steps completed by the last cc_advance
    bool budget_on;  // the conservation budget is tracked (cc_set_budget)
    // several bodies (nb >= 2; the one-body fields above are then unused and m = 0): the
    // bodies, the first vertex of each in the vertex arrays, their total, and the host image
    // of the bodies' block (uploaded after the argument block) with its device address
    int nb;
    std::vector<HostBody> hb;
    std::vector<int> vbase;
    int mtot;
    std::vector<char> hset;
    char* d_set;
    std::string err;
};

struct cc_batch {
    Engine eng;
    hipStream_t stream;
    char* ws;
    std::string err;
};

namespace {

// message of the last failed call without a context (cc_create, cc_totals_state) on this
// thread; cc_last_error(NULL) returns it
thread_local std::string g_create_err;

cc_status fail(cc_ctx* c, cc_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}
cc_status bfail(cc_batch* b, cc_status s, const std::string& msg) {
    if (b) b->err = msg;
    return s;
}

cc_status create_fail(cc_ctx* c, cc_status s, const std::string& msg) {
    g_create_err = msg;
    if (c) cc_destroy(c);
    return s;
}

#define HIPCHK(ctx, expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(ctx, CC_ERR_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)
#define BHIPCHK(b, expr)                                                                    \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return bfail(b, CC_ERR_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
T* at(cc_ctx* c, size_t off) {
    return reinterpret_cast<T*>(c->ws + off);
}

bool fp32(const cc_ctx* c) { return c->cfg.precision == CC_FP32_GEOM64; }

// Rigid pose at time t: rotation by theta(t) about the body-frame origin, then the origin
// at ref + v t.  The device poses with the same formula from (cs, sn, cx, cy).
Pose pose_at(const cc_ctx* c, double t) {
    double th = c->theta0 + c->amp * std::sin(c->omega * t);
    return Pose{std::cos(th), std::sin(th), c->ref_x + c->vx * t, c->ref_y + c->vy * t};
}
void pose_xy(const cc_ctx* c, const Pose& px, const Pose& py, double* out) {
    for (int k = 0; k < c->m; k++) {
        double bx = c->bverts[2 * k], by = c->bverts[2 * k + 1];
        out[2 * k] = (px.cs * bx - px.sn * by) + px.cx;
        out[2 * k + 1] = (py.sn * bx + py.cs * by) + py.cy;
    }
}

// Certificate discs of a posed convex polygon pv (m >= 8): about the vertex centroid, a
// disc inside the polygon (radius: the least distance to an edge line) and one containing
// it (the largest vertex distance), shrunk and grown by a relative 1e-6 (Cert); none when
// the polygon is too thin for them to help.
Cert poly_cert(const double* pv, int m) {
    Cert q{0.0, 0.0, -1.0, 0.0};
    if (m < 8) return q;
    double sx = 0.0, sy = 0.0;
    for (int k = 0; k < m; k++) {
        sx += pv[2 * k];
        sy += pv[2 * k + 1];
    }
    double cx = sx / m, cy = sy / m;
    double rin = INFINITY, rr = 0.0;
    for (int k = 0; k < m; k++) {
        int k1 = k + 1 == m ? 0 : k + 1;
        double ex = pv[2 * k1] - pv[2 * k], ey = pv[2 * k1 + 1] - pv[2 * k + 1];
        double l2 = ex * ex + ey * ey;
        if (l2 > 0.0) rin = std::min(rin, (ex * (cy - pv[2 * k + 1]) - ey * (cx - pv[2 * k])) / std::sqrt(l2));
        double dx = pv[2 * k] - cx, dy = pv[2 * k + 1] - cy;
        rr = std::max(rr, dx * dx + dy * dy);
    }
    double rout = std::sqrt(rr);
    if (rin > 1e-7 * rout && std::isfinite(rin)) {
        q.cx = cx;
        q.cy = cy;
        q.rin2 = (rin * (1.0 - 1e-6)) * (rin * (1.0 - 1e-6));
        q.rout2 = (rout * (1.0 + 1e-6)) * (rout * (1.0 + 1e-6));
    }
    return q;
}

// Extremes of a polygon (first vertices attaining them, as a sequential scan with strict
// comparisons finds them).
Extremes body_extremes(const double* pv, int m) {
    Extremes X{pv[0], pv[0], pv[1], pv[1], 0.0, 0, 0, 0, 0};
    for (int k = 1; k < m; k++) {
        if (pv[2 * k] < X.xlo) X.xlo = pv[2 * k], X.il = k;
        if (pv[2 * k] > X.xhi) X.xhi = pv[2 * k], X.ir = k;
        if (pv[2 * k + 1] < X.ylo) X.ylo = pv[2 * k + 1], X.ib = k;
        if (pv[2 * k + 1] > X.yhi) X.yhi = pv[2 * k + 1], X.it = k;
    }
    X.mag = std::max(std::max(std::fabs(X.xlo), std::fabs(X.xhi)), std::max(std::fabs(X.ylo), std::fabs(X.yhi)));
    return X;
}

// Bounding box, certificate discs and cell box of a polygon posed with x from pose px and
// y from pose py.  A body that does not turn is only translated from step to step, which
// moves its discs with it: their radii and the centroid's offset from the pose origin are
// computed once (the rounding of the posed coordinates, ~1e-16 of their size, stays far
// inside the 1e-6 margins); a turning body's discs are computed from its posed vertices.
void poly_info(const cc_ctx* c, const double* pv, const Pose& px, const Pose& py, Poly& P, Box& cells) {
    int m = c->m;
    P.m = m;
    if (c->amp == 0.0) {  // translated: the turned body's extremes plus the translation
        const Extremes& X = c->ext0;
        P.xmin = X.xlo + px.cx;
        P.xmax = X.xhi + px.cx;
        P.ymin = X.ylo + py.cy;
        P.ymax = X.yhi + py.cy;
        P.il = X.il;
        P.ir = X.ir;
        P.ib = X.ib;
        P.it = X.it;
    } else {
        P.xmin = P.ymin = INFINITY;
        P.xmax = P.ymax = -INFINITY;
        for (int k = 0; k < m; k++) {
            P.xmin = std::fmin(P.xmin, pv[2 * k]);
            P.xmax = std::fmax(P.xmax, pv[2 * k]);
            P.ymin = std::fmin(P.ymin, pv[2 * k + 1]);
            P.ymax = std::fmax(P.ymax, pv[2 * k + 1]);
        }
        P.ib = P.it = P.il = P.ir = 0;
        for (int k = 1; k < m; k++) {
            if (pv[2 * k + 1] < pv[2 * P.ib + 1]) P.ib = k;
            if (pv[2 * k + 1] > pv[2 * P.it + 1]) P.it = k;
            if (pv[2 * k] < pv[2 * P.il]) P.il = k;
            if (pv[2 * k] > pv[2 * P.ir]) P.ir = k;
        }
    }
    Cert q = c->amp == 0.0 ? c->cert0 : poly_cert(pv, m);
    if (c->amp == 0.0 && q.rin2 >= 0.0) {
        q.cx += px.cx;
        q.cy += py.cy;
    }
    P.cx = q.cx;
    P.cy = q.cy;
    P.rin2 = q.rin2;
    P.rout2 = q.rout2;
    cells = m == 0 ? Box{0, 0, 0, 0}
                   : cells_of_bbox(P.xmin, P.xmax, P.ymin, P.ymax, c->cfg.x_lo, c->cfg.x_hi, c->cfg.y_lo,
                                   c->cfg.y_hi, c->hx, c->hy, c->g.nx, c->g.ny);
}

bool has_body(const cc_ctx* c) { return c->m > 0 || c->nb > 1; }

BodySet* hset_of(cc_ctx* c) { return reinterpret_cast<BodySet*>(c->hset.data()); }

// Body b of several, posed with its x coordinates at time tx and its y coordinates at ty
// (the stage polygon of a split step mixes the two; tx = ty: the body at that time), with
// the one-body formula.
void body_pose_xy(const cc_ctx* c, int b, double tx, double ty, double* out) {
    const HostBody& B = c->hb[b];
    double thx = B.theta0 + B.amp * std::sin(B.omega * tx), thy = B.theta0 + B.amp * std::sin(B.omega * ty);
    double csx = std::cos(thx), snx = std::sin(thx), csy = std::cos(thy), sny = std::sin(thy);
    double cx = B.ref_x + B.vx * tx, cy = B.ref_y + B.vy * ty;
    int m = (int)B.verts.size() / 2;
    for (int k = 0; k < m; k++) {
        double bx = B.verts[2 * k], by = B.verts[2 * k + 1];
        out[2 * k] = (csx * bx - snx * by) + cx;
        out[2 * k + 1] = (sny * bx + csy * by) + cy;
    }
}

// Level slot `slot` of several bodies posed with x at tx and y at ty: posed vertices and
// polygons (bounding boxes; no certificate discs) into the host image of the bodies' block.
// Returns the union of the bodies' cell boxes.
Box bodies_level(cc_ctx* c, int slot, double tx, double ty) {
    BodySet* S = hset_of(c);
    double* V = reinterpret_cast<double*>(c->hset.data() + SET_VERTS) + 2 * (size_t)slot * c->mtot;
    const double* dV = reinterpret_cast<const double*>(c->d_set + SET_VERTS) + 2 * (size_t)slot * c->mtot;
    Box cells{0, 0, 0, 0};
    for (int b = 0; b < c->nb; b++) {
        int m = (int)c->hb[b].verts.size() / 2;
        double* pv = V + 2 * (size_t)c->vbase[b];
        body_pose_xy(c, b, tx, ty, pv);
        Poly P{};
        P.v = dV + 2 * (size_t)c->vbase[b];
        P.m = m;
        P.rin2 = -1.0;
        P.xmin = P.ymin = INFINITY;
        P.xmax = P.ymax = -INFINITY;
        for (int k = 0; k < m; k++) {
            P.xmin = std::fmin(P.xmin, pv[2 * k]);
            P.xmax = std::fmax(P.xmax, pv[2 * k]);
            P.ymin = std::fmin(P.ymin, pv[2 * k + 1]);
            P.ymax = std::fmax(P.ymax, pv[2 * k + 1]);
        }
        S->poly[slot][b] = P;
        cells = box_union(cells, cells_of_bbox(P.xmin, P.xmax, P.ymin, P.ymax, c->cfg.x_lo, c->cfg.x_hi, c->cfg.y_lo,
                                               c->cfg.y_hi, c->hx, c->hy, c->g.nx, c->g.ny));
    }
    return cells;
}

// Each body's rigid map over the step from t0 to t1 and its velocity at mid-step.
void bodies_motion(cc_ctx* c, double t0, double t1) {
    BodySet* S = hset_of(c);
    double th = t0 + 0.5 * (t1 - t0);
    for (int b = 0; b < c->nb; b++) {
        const HostBody& B = c->hb[b];
        double th0 = B.theta0 + B.amp * std::sin(B.omega * t0);
        double th1 = B.theta0 + B.amp * std::sin(B.omega * t1);
        Motion& M = S->mot[b];
        M.cosd = std::cos(th1 - th0);
        M.sind = std::sin(th1 - th0);
        M.c0x = B.ref_x + B.vx * t0;
        M.c0y = B.ref_y + B.vy * t0;
        M.c1x = B.ref_x + B.vx * t1;
        M.c1y = B.ref_y + B.vy * t1;
        M.vx = B.vx;
        M.vy = B.vy;
        M.thd = B.amp * B.omega * std::cos(B.omega * th);
        M.chx = B.ref_x + B.vx * th;
        M.chy = B.ref_y + B.vy * th;
    }
}

bool geo_fits(const cc_ctx* c, const Box& r) { return box_empty(r) || (r.w() <= c->lay.gw && r.h() <= c->lay.gh); }

unsigned nblk(size_t n, int t) { return (unsigned)((n + t - 1) / t); }
unsigned nblk(size_t n) { return nblk(n, TPB); }

// An event pair of kind `kind` (0 dense x, 1 dense y, 2 box phases, 3 geometry) from the
// engine's spares, recorded as pending.
TimedPair engine_pair(Engine& E, int kind) {
    if (E.pool.empty()) {
        TimedPair p;
        (void)hipEventCreate(&p.a);
        (void)hipEventCreate(&p.b);
        E.pool.push_back(p);
    }
    TimedPair tp = E.pool.back();
    E.pool.pop_back();
    tp.kind = kind;
    E.pending.push_back(tp);
    return tp;
}

void tstart(cc_ctx* c, int kind, TimedPair& tp) {
    if (!(c->eng.timing & 2)) return;
    tp = engine_pair(c->eng, kind);
    (void)hipEventRecord(tp.a, c->stream);
}
void tstop(cc_ctx* c, TimedPair& tp) {
    if (!(c->eng.timing & 2)) return;
    (void)hipEventRecord(tp.b, c->stream);
}

// Several bodies: no vertex of any body moves a cell or more over the step from t0 to t1.
cc_status bodies_check_motion(cc_ctx* c, double t0, double t1) {
    for (int b = 0; b < c->nb; b++) {
        size_t n = c->hb[b].verts.size();
        std::vector<double> p0(n), p1(n);
        body_pose_xy(c, b, t0, t0, p0.data());
        body_pose_xy(c, b, t1, t1, p1.data());
        for (size_t k = 0; k < n; k += 2)
            if (!(std::fabs(p1[k] - p0[k]) < c->hx) || !(std::fabs(p1[k + 1] - p0[k + 1]) < c->hy))
                return fail(c, CC_ERR_MOTION, "a body moves a cell or more within one sweep");
    }
    return CC_OK;
}

cc_status check_motion(cc_ctx* c, const std::vector<double>& p0, const std::vector<double>& p1) {
    for (int k = 0; k < c->m; k++) {
        double dx = std::fabs(p1[2 * k] - p0[2 * k]), dy = std::fabs(p1[2 * k + 1] - p0[2 * k + 1]);
        if (!(dx < c->hx) || !(dy < c->hy))
            return fail(c, CC_ERR_MOTION, "the body moves a cell or more within one sweep");
    }
    return CC_OK;
}

// Blocks of a geometry or aperture stage launch of one context (0 without a body): one
// thread per item of the capacity, at most GEO_BLOCK_CAP blocks per level job (a larger
// region takes several passes: capacities follow the body's circumscribed circle, which
// for a long body is far larger than its box), and for a many-sided body at least about
// one wavefront per boundary item of the region (those take a wavefront's chain search
// each); the geometry stages run both level jobs side by side, each on its own half.  The
// face stage takes twice the cap of the others (measured on the 4096 x 4096 aerofoil, whose
// blocks each stage a 1024-sided polygon); with several bodies (no polygon staged per
// block, regions up to the whole grid) the cap is higher.
constexpr size_t GEO_BLOCK_CAP = 256, GEO_BLOCK_CAP_FACES = 512, GEO_BLOCK_CAP_BODIES = 2048;
enum GeoStage { GEO_VERTS, GEO_FACES, GEO_CELLS, GEO_SWEPT };
int geo_blocks(const cc_ctx* c, GeoStage st) {
    const Layout& L = c->lay;
    if (!has_body(c)) return 0;
    size_t items;
    switch (st) {
        case GEO_VERTS: items = (size_t)(L.gw + 1) * (L.gh + 1); break;
        case GEO_FACES: items = (size_t)(L.gw + 1) * L.gh + (size_t)L.gw * (L.gh + 1); break;
        case GEO_CELLS: items = (size_t)L.gw * L.gh; break;
        default: items = std::max((size_t)(L.capw + 1) * L.caph, (size_t)L.capw * (L.caph + 1)); break;
    }
    size_t walkers = c->m > SMALL_POLY ? std::min<size_t>(256, (size_t)(L.gw + L.gh)) : 0;
    size_t most = c->nb > 1 ? GEO_BLOCK_CAP_BODIES : (st == GEO_FACES ? GEO_BLOCK_CAP_FACES : GEO_BLOCK_CAP);
    int b = (int)std::max<size_t>(std::min<size_t>(nblk(items, T_WIDE), most), walkers);
    return st == GEO_SWEPT ? b : 2 * b;
}

// ------------------------------------------------------------------ argument blocks
// Constant part of an instance's arguments (pointers into its workspace).
void base_args(cc_ctx* c, StepArgs& a) {
    std::memset(&a, 0, sizeof(a));
    a.g = c->g;
    Stage& S = a.S;
    S.Q = at<double>(c, c->lay.off_sQ);
    S.U1 = at<double>(c, c->lay.off_sU1);
    S.has = at<int8_t>(c, c->lay.off_shas);
    S.bt = at<double>(c, c->lay.off_sbt[0]);
    S.wall = at<int8_t>(c, c->lay.off_swall);
    S.fb = at<double>(c, c->lay.off_sfb);
    S.wv = at<double>(c, c->lay.off_swv);
    S.ahat = at<double>(c, c->lay.off_sahat);
    S.U2 = at<double>(c, c->lay.off_sU2);
    S.gone = at<int8_t>(c, c->lay.off_sgone);
    S.f1 = at<int8_t>(c, c->lay.off_sf1);
    S.f2 = at<int8_t>(c, c->lay.off_sf2);
    S.nbad = at<unsigned int>(c, c->lay.off_nbad);
    S.cap = (int)std::max<size_t>(c->lay.cap, 1);
    a.C.qb = at<double>(c, c->lay.off_qb);
    a.C.stamp = at<int32_t>(c, c->lay.off_stamp);
    a.status = at<unsigned int>(c, c->lay.off_status);
    a.ncol = at<unsigned int>(c, c->lay.off_ncol);
    for (int k = 0; k < 2; k++) {
        a.bt[k] = at<double>(c, c->lay.off_sbt[k]);
    }
    a.cfl_out = at<unsigned long long>(c, c->lay.off_cflout);
    a.nb_cells = geo_blocks(c, GEO_CELLS);
    a.nb_swept = geo_blocks(c, GEO_SWEPT);
    a.spd = at<unsigned long long>(c, c->lay.off_spd);
    a.spd_dense = c->lay.spd_dense;
    a.bs.base = c->budget_on ? at<double>(c, c->lay.off_bslot) : nullptr;
    a.bs.patch = c->lay.bs_patch;
    a.bs.cover = c->lay.bs_cover;
    a.budget = at<double>(c, c->lay.off_budget);
    for (int k = 0; k < 2; k++) {
        GeoJob& J = a.geo[k];
        J.body = at<double>(c, c->lay.off_body);
    }
}

void set_geo(cc_ctx* c, GeoJob& J, int slot, const Box& reg, const Pose& px, const Pose& py) {
    J.L = c->lev[slot];
    J.reg = reg;
    J.cs_x = px.cs;
    J.sn_x = px.sn;
    J.cx_x = px.cx;
    J.cs_y = py.cs;
    J.sn_y = py.sn;
    J.cy_y = py.cy;
    J.active = has_body(c) && !box_empty(reg);
}

Box sweep_box(cc_ctx* c, const Box& a, const Box& b) { return sweep_box_of(a, b, c->g.nx, c->g.ny); }

void set_sweep(cc_ctx* c, SweepJob& J, int s, double dt) {
    int first = s == 0;
    int sl = first ? c->s0 : c->sm, el = first ? c->sm : c->s1;
    J.Ls = c->lev[sl];
    J.Le = c->lev[el];
    J.B = sweep_box(c, c->lbox[sl], c->lbox[el]);
    J.dir = first ? c->parity : 1 - c->parity;
    J.first = first;
    J.lam = dt / (J.dir == 0 ? c->hx : c->hy);
    int rin = first ? c->cur : 1 - c->cur;
    J.Uin = c->ws + c->lay.off_u[rin];
    J.Uout = c->ws + c->lay.off_u[1 - rin];
}

// Host part of a step: poses, level boxes, regions, sweep boxes and motion; fills the
// instance's argument block.  The context's level bookkeeping is updated as if the step's
// geometry had run (the launches follow in stream order).
cc_status prepare_step(cc_ctx* c, double dt, StepArgs& a) {
    if (!c->have_state) return fail(c, CC_ERR_ARG, "no state set");
    if (c->in_step) return fail(c, CC_ERR_ARG, "step already begun");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, CC_ERR_MOTION, "dt must be positive");
    double t1 = c->t + dt;
    base_args(c, a);
    if (c->nb > 1) {
        // several bodies, posed on the host: the stage level (the first sweep's coordinate
        // at t^{n+1}, the other at t^n) and the end level, and each body's motion
        cc_status st = bodies_check_motion(c, c->t, t1);
        if (st != CC_OK) return st;
        Box cm = c->parity == 0 ? bodies_level(c, c->sm, t1, c->t) : bodies_level(c, c->sm, c->t, t1);
        Box c1 = bodies_level(c, c->s1, t1, t1);
        Box rm = box_union(c->lbox[c->sm], cm), r1 = box_union(c->lbox[c->s1], c1);
        c->lbox[c->sm] = cm;
        c->lbox[c->s1] = c1;
        Pose z{1.0, 0.0, 0.0, 0.0};
        set_geo(c, a.geo[0], c->sm, rm, z, z);
        set_geo(c, a.geo[1], c->s1, r1, z, z);
        bodies_motion(c, c->t, t1);
        a.bmot = reinterpret_cast<const Motion*>(c->d_set + offsetof(BodySet, mot));
    } else if (c->m > 0) {
        int m = c->m;
        Pose q0 = pose_at(c, c->t), q1 = pose_at(c, t1);
        // stage polygon: the first sweep's coordinate at t^{n+1}, the other at t^n
        Pose mx = c->parity == 0 ? q1 : q0, my = c->parity == 0 ? q0 : q1;
        // a body that does not turn needs its vertices only when its translation is close
        // to a cell (its extremes follow from the turned body's)
        bool turning = c->amp != 0.0;
        bool check = turning || !(surely_within(q0.cx, q1.cx, c->hx, c->ext0.mag) &&
                                  surely_within(q0.cy, q1.cy, c->hy, c->ext0.mag));
        std::vector<double> p1, pm;
        if (check) {
            std::vector<double> p0(2 * m);
            p1.resize(2 * m);
            pose_xy(c, q0, q0, p0.data());
            pose_xy(c, q1, q1, p1.data());
            cc_status st = check_motion(c, p0, p1);
            if (st != CC_OK) return st;
        }
        if (turning) {
            pm.resize(2 * m);
            pose_xy(c, mx, my, pm.data());
        }
        Poly Pm = c->lev[c->sm].poly, P1 = c->lev[c->s1].poly;
        Box cm, c1;
        poly_info(c, turning ? pm.data() : nullptr, mx, my, Pm, cm);
        poly_info(c, turning ? p1.data() : nullptr, q1, q1, P1, c1);
        Box rm = box_union(c->lbox[c->sm], cm), r1 = box_union(c->lbox[c->s1], c1);
        if (!geo_fits(c, rm) || !geo_fits(c, r1)) return fail(c, CC_ERR_WORKSPACE, "geometry region exceeds capacity");
        c->lev[c->sm].poly = Pm;
        c->lev[c->s1].poly = P1;
        c->lbox[c->sm] = cm;
        c->lbox[c->s1] = c1;
        set_geo(c, a.geo[0], c->sm, rm, mx, my);
        set_geo(c, a.geo[1], c->s1, r1, q1, q1);
        // rigid map of the step and the wall velocity at mid-step
        double th0 = c->theta0 + c->amp * std::sin(c->omega * c->t);
        double th1 = c->theta0 + c->amp * std::sin(c->omega * t1);
        Motion& M = c->mot;
        M.cosd = std::cos(th1 - th0);
        M.sind = std::sin(th1 - th0);
        M.c0x = c->ref_x + c->vx * c->t;
        M.c0y = c->ref_y + c->vy * c->t;
        M.c1x = c->ref_x + c->vx * t1;
        M.c1y = c->ref_y + c->vy * t1;
        double th = c->t + 0.5 * dt;
        M.vx = c->vx;
        M.vy = c->vy;
        M.thd = c->amp * c->omega * std::cos(c->omega * th);
        M.chx = c->ref_x + c->vx * th;
        M.chy = c->ref_y + c->vy * th;
    }
    a.mot = c->mot;
    for (int s = 0; s < 2; s++) {
        set_sweep(c, a.sw[s], s, dt);
        const Box& B = a.sw[s].B;
        if (!box_empty(B) && ((size_t)B.w() > (size_t)c->lay.capw || (size_t)B.h() > (size_t)c->lay.caph))
            return fail(c, CC_ERR_WORKSPACE, "sweep region exceeds the staging capacity");
    }
    a.step_id = (int32_t)(c->step & 0x7fffffff);
    a.dt = dt;
    c->step_dt = dt;
    c->last_sweep_box = a.sw[1].B;
    return CC_OK;
}

// Geometry-only argument block: the level `slot` posed at time t, in up to two jobs (the
// slot's previous region and the new one, when their union exceeds the capacity).
cc_status prepare_geometry(cc_ctx* c, double t, int slot, StepArgs& a) {
    base_args(c, a);
    if (c->nb > 1) {
        Box cells = bodies_level(c, slot, t, t);
        Pose z{1.0, 0.0, 0.0, 0.0};
        set_geo(c, a.geo[0], slot, box_union(c->lbox[slot], cells), z, z);
        c->lbox[slot] = cells;
        return CC_OK;
    }
    if (c->m == 0) return CC_OK;
    Pose q = pose_at(c, t);
    std::vector<double> pv(2 * c->m);
    pose_xy(c, q, q, pv.data());
    Box cells;
    poly_info(c, pv.data(), q, q, c->lev[slot].poly, cells);
    Box reg = box_union(c->lbox[slot], cells);
    if (geo_fits(c, reg)) {
        set_geo(c, a.geo[0], slot, reg, q, q);
    } else {
        set_geo(c, a.geo[0], slot, c->lbox[slot], q, q);
        set_geo(c, a.geo[1], slot, cells, q, q);
    }
    c->lbox[slot] = cells;
    return CC_OK;
}

// ------------------------------------------------------------------ engine bookkeeping
int units_of(int, int n) { return n; }

// Box launches take at most BOX_BLOCK_CAP blocks of T_BOX cells (BOXW_BLOCK_CAP of T_WIDE,
// PATCH_BLOCK_CAP patch segments or tiles) per member and loop over larger boxes; the persistent mode
// walks the uncapped tables.  Several bodies (boxes up to the whole grid): four times as many.
constexpr int BOX_BLOCK_CAP = 2048, BOXW_BLOCK_CAP = 512, PATCH_BLOCK_CAP = 2048;

int kind_blocks(const cc_ctx* c, const Engine& E, int kind) {
    const Layout& L = c->lay;
    int m = c->m;
    bool capped = E.mode != CC_LAUNCH_PERSISTENT;
    int scale = c->nb > 1 ? 4 : 1;
    auto cap = [&](int b, int most) { return capped ? std::min(b, scale * most) : b; };
    if (!has_body(c) && (kind <= L_BOX || kind == L_CS || kind == L_PX || kind == L_PY)) return 0;
    switch (kind) {
        case L_POSE: return (int)nblk((size_t)m, T_WIDE);
        case L_V1: return geo_blocks(c, GEO_VERTS);
        case L_F1: return geo_blocks(c, GEO_FACES);
        case L_C1: return geo_blocks(c, GEO_CELLS);
        case L_S1: return geo_blocks(c, GEO_SWEPT);
        case L_CS: return geo_blocks(c, GEO_CELLS) + 2 * geo_blocks(c, GEO_SWEPT);
        case L_BOX: return cap((int)nblk(std::max<size_t>(L.cap, 1), T_BOX), BOX_BLOCK_CAP);
        case L_BOXW: return cap((int)nblk(std::max<size_t>(L.cap, 1), T_WIDE), BOXW_BLOCK_CAP);
        case L_PX: return cap(std::max(patch_line_blocks<0>(L.capw, L.caph), 1), PATCH_BLOCK_CAP);
        case L_PY: return cap(std::max(patch_tile_blocks(L.capw, L.caph), 1), PATCH_BLOCK_CAP);
        case L_DX: return dense_blocks(0, E.tile_x, c->g.nx, c->g.ny);
        case L_DY: return dense_blocks(1, E.tile_y, c->g.nx, c->g.ny);
    }
    return 0;
}

void drop_graphs(Engine& E) {
    for (int b = 0; b < 2; b++) {
        if (E.gexec[b]) (void)hipGraphExecDestroy(E.gexec[b]);
        E.gexec[b] = nullptr;
        E.gkey[b] = -1;
    }
    for (auto& g : E.pexec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    for (auto& g : E.pexec_run) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

// Offsets of every launch kind for the current members; uploads them (stream-ordered,
// from pageable memory, so the call returns after the copy has been staged).
// The box's first phase shares a dense launch, where its latency-bound blocks run beside
// the tiles instead of in a launch of their own.  The y kernels hold a column's states in
// registers anyway, so they take it at no cost.  The x kernel alone needs few registers,
// and on large grids the merged kernel's registers (set by the box code) halve the tiles'
// occupancy, which costs more than a launch: the 4096 x 4096 x sweep takes 163 us merged
// against 108 us alone (FP32, 4-row blocks), while the box phase alone takes about 12 us.
constexpr size_t MERGE_WALL_CELLS = (size_t)1 << 21;

hipError_t engine_plan(Engine& E, hipStream_t stream) {
    int n = (int)E.mem.size();
    size_t cells = 0;
    for (const cc_ctx* c : E.mem) cells += (size_t)c->g.nx * c->g.ny;
    E.merge_x = cells <= MERGE_WALL_CELLS;
    int stride = 2 * E.cap_n + 1;
    std::vector<int> all((size_t)NKINDS * stride, 0);
    for (int k = 0; k < NKINDS; k++) {
        int nu = units_of(k, n);
        E.h_off[k].assign(nu + 1, 0);
        for (int u = 0; u < nu; u++) {
            const cc_ctx* c = E.mem[u];
            E.h_off[k][u + 1] = E.h_off[k][u] + kind_blocks(c, E, k);
        }
        std::copy(E.h_off[k].begin(), E.h_off[k].end(), all.begin() + (size_t)k * stride);
    }
    drop_graphs(E);
    hipError_t e = hipMemcpyAsync(E.d_off, all.data(), all.size() * sizeof(int), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    return e;
}

const int* koff(const Engine& E, int kind) { return E.d_off + (size_t)kind * (2 * E.cap_n + 1); }
int ktotal(const Engine& E, int kind) { return E.h_off[kind].empty() ? 0 : E.h_off[kind].back(); }

// Waits for event ev, polling it first: a step's read-back is usually due within a few
// hundred microseconds, and a blocking wait adds the thread's wake-up to every step.
hipError_t wait_event(hipEvent_t ev) {
    for (int k = 0; k < 200000; k++) {
        hipError_t e = hipEventQuery(ev);
        if (e != hipErrorNotReady) return e;
    }
    return hipEventSynchronize(ev);
}

// Waits until host buffer b may be rewritten.
hipError_t engine_hostbuf(Engine& E, int b) {
    if (E.ev_used[b]) return hipEventSynchronize(E.ev[b]);
    return hipSuccess;
}

template <typename K, typename... Args>
void klaunch(K kern, int blocks, int threads, hipStream_t s, Args... args) {
    if (blocks > 0) hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), 0, s, args...);
}

// Geometry of both level jobs of every member: vertex classes (and the posed polygons),
// face intervals, volume fractions.
void launch_geometry(const Engine& E, hipStream_t s) {
    int n = (int)E.mem.size();
    const StepArgs* A = E.d_args;
    if (E.multi) {
        klaunch(kb_geo<0, true>, ktotal(E, L_V1), T_WIDE, s, A, koff(E, L_V1), n);
        klaunch(kb_geo<1, true>, ktotal(E, L_F1), T_WIDE, s, A, koff(E, L_F1), n);
        klaunch(kb_geo<2, true>, ktotal(E, L_C1), T_WIDE, s, A, koff(E, L_C1), n);
        return;
    }
    klaunch(kb_geo<0>, ktotal(E, L_V1), T_WIDE, s, A, koff(E, L_V1), n);
    klaunch(kb_geo<1>, ktotal(E, L_F1), T_WIDE, s, A, koff(E, L_F1), n);
    klaunch(kb_geo<2>, ktotal(E, L_C1), T_WIDE, s, A, koff(E, L_C1), n);
}

// Dense launches of sweep sw: bit 0 of `which` the x-sweep kernel, bit 1 the y-sweep
// kernel (a member's direction in this sweep picks which one does its work).  ta/tb:
// events recorded by the launch itself around its execution (one kernel only), or null.
// wall: the first of these launches also runs the box cells' first phase (donations and
// wall quantities) in blocks of its own ahead of the tiles.
template <typename R>
void launch_dense(const Engine& E, hipStream_t s, int sw, int which, hipEvent_t ta, hipEvent_t tb, int fold = 0,
                  bool wall = false) {
    int n = (int)E.mem.size();
    const StepArgs* A = E.d_args;
    int nwall = wall ? ktotal(E, L_BOXW) : 0;
    const int* ow = koff(E, L_BOXW);
    for (int d = 0; d < 2; d++) {
        if (!((which >> d) & 1)) continue;
        int kind = d == 0 ? L_DX : L_DY;
        int blocks = ktotal(E, kind);
        if (blocks == 0) continue;
        const int* off = koff(E, kind);
        auto go = [&](auto kern, auto wkern, int threads) {
            if (nwall > 0) {  // the box blocks ahead of the tiles in one launch
                if (ta)
                    hipExtLaunchKernelGGL(wkern, dim3(nwall + blocks), dim3(threads), 0, s, ta, tb, 0, A, ow, nwall, off,
                                          n, sw, fold);
                else
                    hipLaunchKernelGGL(wkern, dim3(nwall + blocks), dim3(threads), 0, s, A, ow, nwall, off, n, sw,
                                       fold);
                nwall = 0;
            } else if (ta) {
                hipExtLaunchKernelGGL(kern, dim3(blocks), dim3(threads), 0, s, ta, tb, 0, A, off, n, sw, fold);
            } else {
                hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), 0, s, A, off, n, sw, fold);
            }
        };
        if (d == 0) {
            switch (E.tile_x) {
                case 0: go(kb_dense_x<R, 1>, kb_wall_dense_x<R, 1>, DX_T); break;
                case 1: go(kb_dense_x<R, 2>, kb_wall_dense_x<R, 2>, DX_T); break;
                case 2: go(kb_dense_x<R, 4>, kb_wall_dense_x<R, 4>, DX_T); break;
                default: go(kb_dense_x<R, 8>, kb_wall_dense_x<R, 8>, DX_T); break;
            }
        } else {
            switch (E.tile_y) {
                case 0: go(kb_dense_y<R, 8>, kb_wall_dense_y<R, 8>, 256); break;
                case 1: go(kb_dense_y<R, 12>, kb_wall_dense_y<R, 12>, 256); break;
                case 4: go(kb_dense_yc<R, 4>, kb_wall_dense_yc<R, 4>, DYC_T); break;
                case 5: go(kb_dense_yc<R, 8>, kb_wall_dense_yc<R, 8>, DYC_T); break;
                default:
                    if constexpr (sizeof(R) == 4) {
                        if (E.tile_y == 2) go(kb_dense_y<R, 16>, kb_wall_dense_y<R, 16>, 256);
                        else go(kb_dense_y<R, 24>, kb_wall_dense_y<R, 24>, 256);
                    }
                    break;
            }
        }
    }
    if (wall && nwall > 0)  // no dense launch took the box blocks
        klaunch(kb_stagewall<R>, ktotal(E, L_BOX), T_BOX, s, A, koff(E, L_BOX), n, sw);
}

// The box phase's first launch of its own (several bodies: the kernel that takes each wall
// cell's body).
template <typename R>
void launch_stagewall(const Engine& E, hipStream_t s, int sw) {
    int n = (int)E.mem.size();
    if (E.multi) klaunch(kb_stagewall<R, true>, ktotal(E, L_BOX), T_BOX, s, E.d_args, koff(E, L_BOX), n, sw);
    else klaunch(kb_stagewall<R>, ktotal(E, L_BOX), T_BOX, s, E.d_args, koff(E, L_BOX), n, sw);
}

// The dense launches of sweep sw (`which` as for launch_dense) with the box cells' first
// phase placed as engine_plan decided.  ta/tb (nullable): event pairs of the x and y
// launches, from tp(d).
template <typename R, class TP>
void launch_sweep_dense(const Engine& E, hipStream_t s, int sw, int which, int fold, TP&& tp) {
    bool wall_y = (which & 2) != 0 && !E.multi, wall_x = !wall_y && E.merge_x && !E.multi;
    if (!wall_x && !wall_y) launch_stagewall<R>(E, s, sw);
    for (int d = 0; d < 2; d++) {
        if (!((which >> d) & 1)) continue;
        TimedPair p = tp(d);
        launch_dense<R>(E, s, sw, 1 << d, p.a, p.b, fold, d == 0 ? wall_x : wall_y);
    }
}

// Box phases before the dense sweep.
template <typename R>
void launch_box_pre(const Engine& E, hipStream_t s, int sw, bool swept = true) {
    int n = (int)E.mem.size();
    const StepArgs* A = E.d_args;
    if (swept && E.multi) klaunch(kb_swept<true>, ktotal(E, L_S1), T_WIDE, s, A, koff(E, L_S1), n, sw);
    else if (swept) klaunch(kb_swept<>, ktotal(E, L_S1), T_WIDE, s, A, koff(E, L_S1), n, sw);
    launch_stagewall<R>(E, s, sw);
}
// Box phases after the dense sweep (`which` as for the dense launches): patch update,
// covering, both collapse rounds.  last: the sweep ends a captured step; covering leaves the
// box cells' wave-speed partials and the collapse launch combines the member's partials.
template <typename R>
void launch_box_post(const Engine& E, hipStream_t s, int sw, int which, int last = 0) {
    int n = (int)E.mem.size();
    const StepArgs* A = E.d_args;
    int nb = ktotal(E, L_BOX);
    const int* ob = koff(E, L_BOX);
    if (which & 1) klaunch(kb_patch_lines<0, R>, ktotal(E, L_PX), PL_T, s, A, koff(E, L_PX), n, sw);
    if (which & 2) klaunch(kb_patch_tiles<R>, ktotal(E, L_PY), PT_T, s, A, koff(E, L_PY), n, sw);
    klaunch(kb_cover<R>, nb, T_BOX, s, A, ob, n, sw, last);
    klaunch(kb_fix_block<R>, n, T_FIX, s, E.d_args, koff(E, L_DX), koff(E, L_DY), ob, sw, last, E.d_gather);
}

hipError_t engine_upload(Engine& E, hipStream_t s, int b) {
    return hipMemcpyAsync(E.d_args, E.h_args[b], E.mem.size() * sizeof(StepArgs) + E.extra, hipMemcpyHostToDevice,
                          s);
}

hipError_t engine_alloc_host(Engine& E) {
    hipError_t e = hipSuccess;
    for (int b = 0; b < 2 && e == hipSuccess; b++) {
        e = hipHostMalloc((void**)&E.h_args[b], sizeof(StepArgs) * E.cap_n + E.extra, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&E.ev[b], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipHostMalloc((void**)&E.h_cflout, 24 * (size_t)E.cap_n, hipHostMallocDefault);
    if (e == hipSuccess) E.h_gather = (unsigned int*)(E.h_cflout + 2 * (size_t)E.cap_n);
    int dev = 0, khz = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    E.wait_ticks = (unsigned long long)(khz > 0 ? khz : 100000) * 250ull;  // a quarter of a second
    return e;
}

void engine_free(Engine& E) {
    drop_graphs(E);
    for (auto* v : {&E.pending, &E.pool})
        for (auto& p : *v) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
    E.pending.clear();
    E.pool.clear();
    for (int b = 0; b < 2; b++) {
        if (E.h_args[b]) (void)hipHostFree(E.h_args[b]);
        if (E.ev[b]) (void)hipEventDestroy(E.ev[b]);
        E.h_args[b] = nullptr;
        E.ev[b] = nullptr;
    }
    if (E.h_cflout) (void)hipHostFree(E.h_cflout);
    E.h_cflout = nullptr;
    E.h_gather = nullptr;
}

// One persistent launch of sweep `sw` (tile variants: 1 or 2 rows per x tile, 8 or 12 rows
// per y tile).  The grid is what the device keeps resident at once, so that every block of
// the launch runs concurrently (the barriers between phases rely on it).
template <typename R, int RB, int TR>
hipError_t persist_one(const Engine& E, hipStream_t s, int sw) {
    static int grid = -1;
    if (grid < 0) {
        int per = 0, dev = 0, cus = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kb_sweep<R, RB, TR>, 256, 0);
        if (e == hipSuccess) e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        if (per < 1 || cus < 1) return hipErrorLaunchOutOfResources;
        grid = per * cus;
    }
    PArgs p;
    p.A = E.d_args;
    p.off = E.d_off;
    p.n = (int)E.mem.size();
    p.stride = 2 * E.cap_n + 1;
    p.gs = E.d_sync;
    p.gather = E.d_gather;
    p.wait_ticks = E.wait_ticks;
    p.s = sw;
    hipLaunchKernelGGL((kb_sweep<R, RB, TR>), dim3(grid), dim3(256), 0, s, p);
    return hipGetLastError();
}

bool persist_ok(const Engine& E) {
    return E.mode == 1 && E.tile_x >= 0 && E.tile_x <= 1 && E.tile_y >= 0 && E.tile_y <= 1;
}

template <typename R>
hipError_t launch_persist(const Engine& E, hipStream_t s, int sw) {
    switch (E.tile_x * 2 + E.tile_y) {
        case 0: return persist_one<R, 1, 8>(E, s, sw);
        case 1: return persist_one<R, 1, 12>(E, s, sw);
        case 2: return persist_one<R, 2, 8>(E, s, sw);
        default: return persist_one<R, 2, 12>(E, s, sw);
    }
}

// Whole step of every member, argument blocks in host buffer b, as captured into a graph:
// upload; one persistent launch per sweep (or, for tile variants without one, every phase
// as its own launch); then the read-back of the wave speeds and status words into pinned
// host memory.  dir0: the single member's first direction (only its dense kernels are
// launched on the per-phase path), or -1.
// The geometry launches of a whole step: vertex classes, face intervals, then volume
// fractions with both sweeps' time-averaged apertures.
void launch_geo_step(const Engine& E, hipStream_t s) {
    int n = (int)E.mem.size();
    const StepArgs* A = E.d_args;
    if (E.multi) {
        klaunch(kb_geo<0, true>, ktotal(E, L_V1), T_WIDE, s, A, koff(E, L_V1), n);
        klaunch(kb_geo<1, true>, ktotal(E, L_F1), T_WIDE, s, A, koff(E, L_F1), n);
        klaunch(kb_geo_cells_swept<true>, ktotal(E, L_CS), T_WIDE, s, A, koff(E, L_CS), n);
        return;
    }
    klaunch(kb_geo<0>, ktotal(E, L_V1), T_WIDE, s, A, koff(E, L_V1), n);
    klaunch(kb_geo<1>, ktotal(E, L_F1), T_WIDE, s, A, koff(E, L_F1), n);
    klaunch(kb_geo_cells_swept<>, ktotal(E, L_CS), T_WIDE, s, A, koff(E, L_CS), n);
}

// The axisymmetric source before the step's first sweep (one instance).
template <typename R>
void launch_axisym(const Engine& E, hipStream_t s) {
    if (E.axisym) klaunch(k_axisym<R>, E.axi_blocks, 256, s, (const StepArgs*)E.d_args);
}

// The per-phase launches of a whole step (arguments already in device memory).
template <typename R>
void step_kernels(const Engine& E, hipStream_t s, int dir0) {
    int which0 = dir0 < 0 ? 3 : 1 << dir0, which1 = dir0 < 0 ? 3 : 1 << (1 - dir0);
    int n = (int)E.mem.size();
    const StepArgs* A = E.d_args;
    launch_geo_step(E, s);
    launch_axisym<R>(E, s);
    // the second sweep's dense tiles and its covering leave partial maxima of the new
    // state's wave speeds; its collapse launch (one block per member) combines them
    for (int sw = 0; sw < 2; sw++) {
        launch_sweep_dense<R>(E, s, sw, sw == 0 ? which0 : which1, sw, [](int) { return TimedPair{nullptr, nullptr, 0}; });
        launch_box_post<R>(E, s, sw, sw == 0 ? which0 : which1, sw);
    }
}

// The same launches one by one, each dense (merged wall + dense) launch bracketed by an
// event pair of its own (timing bit 0): their kernel times are those of the captured step.
// Members that sweep the other way get a launch of the other kernel, timed separately.
template <typename R>
void step_kernels_timed(Engine& E, hipStream_t s, int dir0) {
    int which0 = dir0 < 0 ? 3 : 1 << dir0, which1 = dir0 < 0 ? 3 : 1 << (1 - dir0);
    int n = (int)E.mem.size();
    const StepArgs* A = E.d_args;
    launch_geo_step(E, s);
    launch_axisym<R>(E, s);
    for (int sw = 0; sw < 2; sw++) {
        int which = sw == 0 ? which0 : which1;
        launch_sweep_dense<R>(E, s, sw, which, sw, [&](int d) { return engine_pair(E, d); });
        launch_box_post<R>(E, s, sw, which, sw);
    }
}

template <typename R>
void step_sequence_timed(Engine& E, hipStream_t s, int b, int dir0) {
    int n = (int)E.mem.size();
    (void)engine_upload(E, s, b);
    step_kernels_timed<R>(E, s, dir0);
    (void)hipMemcpyAsync(E.h_cflout, E.d_cflout, 16 * (size_t)E.cap_n + 8 * (size_t)n, hipMemcpyDeviceToHost, s);
}

// Reads and recycles the engine's pending event pairs: per kind (dense x, dense y, box,
// geometry) the summed milliseconds and the count, in out[2 kind], out[2 kind + 1].
hipError_t engine_timing_read(Engine& E, hipStream_t s, double* out, int n) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    double sum[4] = {0, 0, 0, 0}, cnt[4] = {0, 0, 0, 0};
    for (auto& p : E.pending) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, p.a, p.b);
        if (e != hipSuccess) return e;
        sum[p.kind] += ms;
        cnt[p.kind] += 1.0;
        E.pool.push_back(p);
    }
    E.pending.clear();
    for (int k = 0; k < 4 && 2 * k + 1 < n; k++) {
        out[2 * k] = sum[k];
        out[2 * k + 1] = cnt[k];
    }
    return hipSuccess;
}

template <typename R>
void step_sequence(Engine& E, hipStream_t s, int b, int dir0) {
    int n = (int)E.mem.size();
    (void)engine_upload(E, s, b);
    if (persist_ok(E)) {
        (void)launch_persist<R>(E, s, 0);
        (void)launch_persist<R>(E, s, 1);
    } else {
        step_kernels<R>(E, s, dir0);
    }
    (void)hipMemcpyAsync(E.h_cflout, E.d_cflout, 16 * (size_t)E.cap_n + 8 * (size_t)n, hipMemcpyDeviceToHost, s);
}

// A device-planned step: its arguments were written on the device (by the planning launch
// for the first step of a run, by the previous step's last block for the others), which
// also plans the next one.  dir0: a single member's first direction, which the host knows
// from the step count alone; -1 for a batch (both dense kernels).
// nsteps: 1, or PLANNED_RUN consecutive steps in one graph (directions alternating from
// dir0; a batch keeps -1): one graph launch, and one gap between graphs, per PLANNED_RUN
// steps.
constexpr int PLANNED_RUN = 4;
template <typename R>
hipError_t engine_planned_step(Engine& E, hipStream_t s, int dir0, int nsteps = 1) {
    if (!s) {  // the null stream cannot be captured: individual launches
        for (int k = 0; k < nsteps; k++) step_kernels<R>(E, s, dir0 < 0 ? -1 : (dir0 + k) & 1);
        return hipGetLastError();
    }
    if (nsteps != 1 && nsteps != PLANNED_RUN) return hipErrorInvalidValue;
    hipGraphExec_t& gx = nsteps == 1 ? E.pexec[dir0 + 1] : E.pexec_run[dir0 + 1];
    if (!gx) {
        hipGraph_t gr;
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        for (int k = 0; k < nsteps; k++) step_kernels<R>(E, s, dir0 < 0 ? -1 : (dir0 + k) & 1);
        e = hipStreamEndCapture(s, &gr);
        if (e != hipSuccess) return e;
        e = hipGraphInstantiate(&gx, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e != hipSuccess) return e;
    }
    return hipGraphLaunch(gx, s);
}

// Launches the captured step graph of host buffer b (capturing it first if needed).
template <typename R>
hipError_t engine_graph_step(Engine& E, hipStream_t s, int b, int dir0) {
    int key = dir0 + 1;
    if (!E.gexec[b] || E.gkey[b] != key) {
        if (E.gexec[b]) (void)hipGraphExecDestroy(E.gexec[b]);
        E.gexec[b] = nullptr;
        hipGraph_t gr;
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        step_sequence<R>(E, s, b, dir0);
        e = hipStreamEndCapture(s, &gr);
        if (e != hipSuccess) return e;
        e = hipGraphInstantiate(&E.gexec[b], gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e != hipSuccess) return e;
        E.gkey[b] = key;
    }
    return hipGraphLaunch(E.gexec[b], s);
}

}  // namespace

extern "C" {

size_t cc_workspace_bytes(const cc_config* cfg, const cc_body* body) {
    if (!cfg || cfg->nx < 1 || cfg->ny < 1) return 0;
    return make_layout(cfg, body).total;
}

size_t cc_workspace_bytes_bodies(const cc_config* cfg, const cc_body* bodies, int32_t nbodies) {
    if (!cfg || cfg->nx < 1 || cfg->ny < 1 || nbodies < 0 || nbodies > CC_MAX_BODIES || (nbodies > 0 && !bodies))
        return 0;
    if (nbodies <= 1) return make_layout(cfg, nbodies == 1 ? bodies : nullptr).total;
    return make_layout(cfg, bodies, nbodies).total;
}

}  // extern "C"

namespace {

// cc_create (nbodies <= 1, body nullable) and cc_create_bodies (nbodies >= 2, body the
// array of bodies).
cc_status create_impl(const cc_config* cfg, const cc_body* body, int nbodies, void* d_ws, size_t ws_bytes,
                      void* hip_stream, cc_ctx** out) {
    if (!out) return create_fail(nullptr, CC_ERR_ARG, "null output pointer");
    *out = nullptr;
    if (!cfg || cfg->nx < 1 || cfg->ny < 1 || !(cfg->x_hi > cfg->x_lo) || !(cfg->y_hi > cfg->y_lo) ||
        !(cfg->gamma > 1.0) || (cfg->options & ~1) != 0 || ((cfg->options & 1) && !(cfg->y_lo >= 0.0)) ||
        (cfg->precision != CC_FP64 && cfg->precision != CC_FP32_GEOM64) ||
        !(cfg->alpha_min >= 0.0 && cfg->alpha_min < 0.5))
        return create_fail(nullptr, CC_ERR_ARG, "invalid configuration");
    for (int k = 0; k < 4; k++)
        if (cfg->bc[k] != CC_BC_TRANSMISSIVE && cfg->bc[k] != CC_BC_REFLECTIVE)
            return create_fail(nullptr, CC_ERR_ARG, "invalid boundary condition");
    bool multi = nbodies > 1;
    for (int b = 0; b < (multi ? nbodies : 1); b++) {
        const cc_body* bd = multi ? &body[b] : body;
        if (bd && bd->nverts > 0 && !bd->verts) return create_fail(nullptr, CC_ERR_ARG, "body without vertices");
        if (bd && bd->nverts > (multi ? BODY_MAX_VERTS : LDS_VERTS))
            return create_fail(nullptr, CC_ERR_UNSUPPORTED,
                               multi ? "one of several bodies with more than 256 vertices"
                                     : "body polygon with more than 2048 vertices");
        if (bd && (bd->nverts > 0 || multi) && !convex_ccw(bd->verts, bd->nverts))
            return create_fail(nullptr, CC_ERR_ARG,
                               "body polygon is not convex and counter-clockwise with 3 or more vertices");
    }
    Layout lay = make_layout(cfg, body, multi ? nbodies : 1);
    if (!d_ws || ws_bytes < lay.total || ((uintptr_t)d_ws % ALIGN) != 0)
        return create_fail(nullptr, CC_ERR_WORKSPACE, "workspace missing, too small or not 256-byte aligned");
    cc_ctx* c = new cc_ctx();
    c->cfg = *cfg;
    c->lay = lay;
    c->ws = (char*)d_ws;
    c->stream = (hipStream_t)hip_stream;
    c->hx = (cfg->x_hi - cfg->x_lo) / (double)cfg->nx;
    c->hy = (cfg->y_hi - cfg->y_lo) / (double)cfg->ny;
    c->g.nx = cfg->nx;
    c->g.ny = cfg->ny;
    for (int k = 0; k < 4; k++) c->g.bc[k] = cfg->bc[k];
    c->g.x_lo = cfg->x_lo;
    c->g.y_lo = cfg->y_lo;
    c->g.hx = c->hx;
    c->g.hy = c->hy;
    c->g.gamma = cfg->gamma;
    c->g.alpha_min = cfg->alpha_min;
    c->m = multi ? 0 : body_m(body);
    c->nb = multi ? nbodies : 0;
    c->mtot = 0;
    c->d_set = nullptr;
    for (int b = 0; b < c->nb; b++) {
        const cc_body& bd = body[b];
        c->hb.push_back(HostBody{std::vector<double>(bd.verts, bd.verts + 2 * (size_t)bd.nverts), bd.ref_x, bd.ref_y,
                                 bd.theta0, bd.vx, bd.vy, bd.pitch_amp, bd.pitch_omega});
        c->vbase.push_back(c->mtot);
        c->mtot += bd.nverts;
    }
    if (multi) {
        c->hset.assign(lay.set_bytes, 0);
        c->d_set = c->ws + lay.off_args + sizeof(StepArgs);
    }
    c->cert0 = Cert{0.0, 0.0, -1.0, 0.0};
    if (c->m > 0) {
        c->bverts.assign(body->verts, body->verts + 2 * c->m);
        c->ref_x = body->ref_x;
        c->ref_y = body->ref_y;
        c->theta0 = body->theta0;
        c->vx = body->vx;
        c->vy = body->vy;
        c->amp = body->pitch_amp;
        c->omega = body->pitch_omega;
        // discs of the body turned by theta0 about the pose origin (not translated)
        Pose q0{std::cos(c->theta0), std::sin(c->theta0), 0.0, 0.0};
        std::vector<double> pv(2 * (size_t)c->m);
        pose_xy(c, q0, q0, pv.data());
        c->cert0 = poly_cert(pv.data(), c->m);
        c->ext0 = body_extremes(pv.data(), c->m);
    }
    c->cur = 0;
    c->s0 = 0;
    c->sm = 1;
    c->s1 = 2;
    c->speeds_ready = false;
    c->speeds_buf = 0;
    c->batch = nullptr;
    c->budget_on = false;
    c->in_step = c->have_state = false;
    c->t = 0.0;
    c->step = 0;
    c->parity = 0;
    c->last_sweep_box = Box{0, 0, 0, 0};
    std::memset(&c->mot, 0, sizeof(c->mot));
    for (int s = 0; s < 3; s++) {
        Level& L = c->lev[s];
        L.vcls = at<int8_t>(c, lay.off_vcls[s]);
        L.fx = at<double2>(c, lay.off_fx[s]);
        L.fy = at<double2>(c, lay.off_fy[s]);
        L.alpha = at<double>(c, lay.off_alpha[s]);
        L.poly = Poly{};
        L.poly.v = at<double>(c, lay.off_poly[s]);
        L.poly.m = 0;
        L.poly.rin2 = -1.0;
        L.parts = nullptr;
        L.np = 0;
        L.cbody = nullptr;
        if (multi) {  // the bodies' polygons of the slot (none posed yet: all fluid)
            L.parts = reinterpret_cast<const Poly*>(c->d_set + offsetof(BodySet, poly)) + (size_t)s * MAX_BODIES;
            L.np = c->nb;
            L.cbody = at<int8_t>(c, lay.off_cbody[s]);
        }
        c->lbox[s] = Box{0, 0, 0, 0};
    }
    // own launch plan (one member)
    Engine& E = c->eng;
    E.prec = cfg->precision;
    E.cap_n = 1;
    E.mem = {c};
    E.d_args = at<StepArgs>(c, lay.off_args);
    E.d_off = at<int>(c, lay.off_offs);
    E.d_cflout = at<unsigned long long>(c, lay.off_cflout);
    E.d_gather = (unsigned int*)(E.d_cflout + 2);
    E.d_sync = at<GridSync>(c, lay.off_sync);
    E.tile_x = 0;  // one row per x-sweep block
    E.tile_y = 0;  // 8-row y-sweep tiles
    E.multi = multi;
    E.extra = lay.set_bytes;
    E.axisym = (cfg->options & 1) != 0;
    E.axi_blocks = (int)std::min<size_t>(nblk(lay.nc, 256), 2048);
    hipError_t e = engine_alloc_host(E);
    if (e != hipSuccess) return create_fail(c, CC_ERR_DEVICE, std::string("host buffers: ") + hipGetErrorString(e));
    // all-fluid levels, clean reductions and lists, stamps that match no step, body vertices
    for (int s = 0; s < 3 && e == hipSuccess; s++) {
        if (e == hipSuccess) e = hipMemsetAsync(c->lev[s].vcls, 0, lay.nvx, c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(c->lev[s].fx, 0, lay.nfx * 16, c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(c->lev[s].fy, 0, lay.nfy * 16, c->stream);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_fill_f64, dim3(nblk(lay.nc)), dim3(TPB), 0, c->stream, (size_t)lay.nc, 1.0,
                               c->lev[s].alpha);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess && has_body(c)) e = hipMemsetAsync(at<int32_t>(c, lay.off_stamp), 0xff, lay.nc * 4, c->stream);
    for (int s = 0; s < 3 && e == hipSuccess && multi; s++) e = hipMemsetAsync(c->lev[s].cbody, 0xff, lay.nc, c->stream);
    if (e == hipSuccess && multi)  // the bodies' block: no body posed yet
        e = hipMemcpyAsync(c->d_set, c->hset.data(), c->hset.size(), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && c->m > 0)
        e = hipMemcpyAsync(at<double>(c, lay.off_body), c->bverts.data(), 16 * (size_t)c->m, hipMemcpyHostToDevice,
                           c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + lay.off_sync, 0, sizeof(GridSync), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + lay.off_nbad, 0, 8, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + lay.off_smax, 0, 16, c->stream);
    // the dense tiles' speed slots start at zero (every combine leaves them so)
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + lay.off_spd, 0, (size_t)16 * NSPD, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + lay.off_status, 0, 4, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + lay.off_ncol, 0, 4, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + lay.off_budget, 0, 16 * 8, c->stream);
    if (e == hipSuccess) e = engine_plan(E, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return create_fail(c, CC_ERR_DEVICE, std::string("initialisation: ") + hipGetErrorString(e));
    *out = c;
    return CC_OK;
}

}  // namespace

extern "C" {

cc_status cc_create(const cc_config* cfg, const cc_body* body, void* d_ws, size_t ws_bytes, void* hip_stream,
                    cc_ctx** out) {
    return create_impl(cfg, body, 1, d_ws, ws_bytes, hip_stream, out);
}

cc_status cc_create_bodies(const cc_config* cfg, const cc_body* bodies, int32_t nbodies, void* d_ws, size_t ws_bytes,
                           void* hip_stream, cc_ctx** out) {
    if (out) *out = nullptr;
    if (nbodies < 0 || nbodies > CC_MAX_BODIES || (nbodies > 0 && !bodies))
        return create_fail(nullptr, CC_ERR_ARG, "between 0 and 4 bodies");
    return create_impl(cfg, nbodies >= 1 ? bodies : nullptr, nbodies > 1 ? nbodies : 1, d_ws, ws_bytes, hip_stream, out);
}

cc_status cc_destroy(cc_ctx* c) {
    if (!c) return CC_ERR_ARG;
    if (c->batch) {
        // leave the batch whatever the removal reports: the batch must never keep a
        // pointer to a destroyed context
        cc_batch* b = c->batch;
        if (cc_batch_remove(b, c) != CC_OK) {
            (void)hipStreamSynchronize(b->stream);
            auto& mem = b->eng.mem;
            mem.erase(std::remove(mem.begin(), mem.end(), c), mem.end());
            c->batch = nullptr;
            (void)engine_plan(b->eng, b->stream);
        }
    }
    (void)hipStreamSynchronize(c->stream);
    engine_free(c->eng);
    delete c;
    return CC_OK;
}

const char* cc_last_error(const cc_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

}  // extern "C"

namespace {

// Uploads argument block `a` through the context's next host buffer.
cc_status own_upload(cc_ctx* c, const StepArgs& a) {
    Engine& E = c->eng;
    int b = E.buf;
    HIPCHK(c, engine_hostbuf(E, b));
    E.h_args[b][0] = a;
    if (E.extra) std::memcpy(reinterpret_cast<char*>(E.h_args[b]) + sizeof(StepArgs), c->hset.data(), E.extra);
    HIPCHK(c, engine_upload(E, c->stream, b));
    HIPCHK(c, hipEventRecord(E.ev[b], c->stream));
    E.ev_used[b] = true;
    E.buf = 1 - b;
    return CC_OK;
}

cc_status geometry_at(cc_ctx* c, double t, int slot) {
    c->speeds_ready = false;
    StepArgs a;
    cc_status st = prepare_geometry(c, t, slot, a);
    if (st != CC_OK) return st;
    if (!has_body(c)) return CC_OK;
    if ((st = own_upload(c, a)) != CC_OK) return st;
    TimedPair tp{};
    tstart(c, 3, tp);
    launch_geometry(c->eng, c->stream);
    tstop(c, tp);
    HIPCHK(c, hipGetLastError());
    return CC_OK;
}

// After the clock or the state is set: the current level is built at t, and so are the two
// other level slots (a step rebuilds a slot over its previous cut-cell box joined with the
// new one, and boxes left from another time, such as those of an earlier run of the same
// context, would make that union exceed the region capacity).
cc_status levels_at(cc_ctx* c, double t) {
    cc_status st = geometry_at(c, t, c->s0);
    for (int k = 0; k < 3 && st == CC_OK; k++)
        if (k != c->s0 && !box_empty(c->lbox[k])) st = geometry_at(c, t, k);
    return st;
}

cc_status not_in_batch(cc_ctx* c) {
    if (c->batch) return fail(c, CC_ERR_ARG, "the context is stepped by a batch");
    return CC_OK;
}

}  // namespace

extern "C" {

cc_status cc_geometry(cc_ctx* c, double t, int32_t level) {
    if (!c || level < 0 || level > 2) return fail(c, CC_ERR_ARG, "bad level");
    if (c->in_step) return fail(c, CC_ERR_ARG, "cc_geometry inside a step");
    int slot = level == 0 ? c->s0 : level == 1 ? c->sm : c->s1;
    return geometry_at(c, t, slot);
}

cc_status cc_geometry_dump(cc_ctx* c, int32_t level, int8_t* d_vcls, double* d_alpha, double* d_bx, double* d_by,
                           int32_t* d_cut, int32_t* d_ncut) {
    if (!c || level < 0 || level > 2) return fail(c, CC_ERR_ARG, "bad level");
    if ((d_cut == nullptr) != (d_ncut == nullptr)) return fail(c, CC_ERR_ARG, "cut list needs both outputs");
    int slot = level == 0 ? c->s0 : level == 1 ? c->sm : c->s1;
    const Level& L = c->lev[slot];
    if (d_cut) {
        const Box& R = c->lbox[slot];
        int cells = box_empty(R) ? 0 : R.w() * R.h();
        if (cells == 0) {
            HIPCHK(c, hipMemsetAsync(d_ncut, 0, sizeof(int32_t), c->stream));
        } else {
            int chunk = (cells + CUT_BLOCKS - 1) / CUT_BLOCKS, nb = (cells + chunk - 1) / chunk;
            int* counts = at<int>(c, c->lay.off_part);  // 4 KiB of the reduction scratch
            CutCells pred{c->g, L};
            hipLaunchKernelGGL(k_list_count<CutCells>, dim3(nb), dim3(CUT_T), 0, c->stream, pred, R, chunk, counts);
            hipLaunchKernelGGL(k_cut_scan, dim3(1), dim3(CUT_T), 0, c->stream, nb, counts, (int*)d_ncut);
            hipLaunchKernelGGL(k_list_write<CutCells>, dim3(nb), dim3(CUT_T), 0, c->stream, pred, R, chunk,
                               (const int*)counts, (int*)d_cut);
        }
    }
    if (d_vcls) HIPCHK(c, hipMemcpyAsync(d_vcls, L.vcls, c->lay.nvx, hipMemcpyDeviceToDevice, c->stream));
    if (d_alpha) HIPCHK(c, hipMemcpyAsync(d_alpha, L.alpha, c->lay.nc * 8, hipMemcpyDeviceToDevice, c->stream));
    if (d_bx)
        hipLaunchKernelGGL(k_interval_beta, dim3(nblk(c->lay.nfx)), dim3(TPB), 0, c->stream, (size_t)c->lay.nfx,
                           (const double2*)L.fx, d_bx);
    if (d_by)
        hipLaunchKernelGGL(k_interval_beta, dim3(nblk(c->lay.nfy)), dim3(TPB), 0, c->stream, (size_t)c->lay.nfy,
                           (const double2*)L.fy, d_by);
    HIPCHK(c, hipGetLastError());
    return CC_OK;
}

cc_status cc_set_state(cc_ctx* c, const double* d_prim, double t0) {
    if (!c || !d_prim) return fail(c, CC_ERR_ARG, "null argument");
    c->speeds_ready = false;
    c->in_step = false;
    c->t = t0;
    c->step = 0;
    c->parity = 0;
    c->cur = 0;
    // the status word starts clear before the level-n geometry (which may set bit 4)
    HIPCHK(c, hipMemsetAsync(c->ws + c->lay.off_status, 0, 4, c->stream));
    cc_status st = levels_at(c, t0);
    if (st != CC_OK) return st;
    const double* al = c->lev[c->s0].alpha;
    if (fp32(c))
        hipLaunchKernelGGL(k_prim_to_u<float>, dim3(nblk(c->lay.nc)), dim3(TPB), 0, c->stream, c->g, al, d_prim,
                           at<float>(c, c->lay.off_u[0]));
    else
        hipLaunchKernelGGL(k_prim_to_u<double>, dim3(nblk(c->lay.nc)), dim3(TPB), 0, c->stream, c->g, al, d_prim,
                           at<double>(c, c->lay.off_u[0]));
    HIPCHK(c, hipMemsetAsync(c->ws + c->lay.off_ncol, 0, 4, c->stream));
    HIPCHK(c, hipMemsetAsync(c->ws + c->lay.off_budget, 0, 16 * 8, c->stream));
    if (has_body(c)) HIPCHK(c, hipMemsetAsync(c->ws + c->lay.off_stamp, 0xff, c->lay.nc * 4, c->stream));
    HIPCHK(c, hipGetLastError());
    c->have_state = true;
    return CC_OK;
}

cc_status cc_set_budget(cc_ctx* c, int32_t on) {
    if (!c || (on != 0 && on != 1)) return fail(c, CC_ERR_ARG, "bad argument");
    if (c->in_step) return fail(c, CC_ERR_ARG, "cc_set_budget inside a step");
    if (on && (c->eng.mode == CC_LAUNCH_PERSISTENT || (c->batch && c->batch->eng.mode == CC_LAUNCH_PERSISTENT)))
        return fail(c, CC_ERR_UNSUPPORTED, "the budget is not tracked in the persistent launch mode");
    HIPCHK(c, hipStreamSynchronize(c->stream));  // captured steps hold the argument blocks of the old setting
    if (c->batch) HIPCHK(c, hipStreamSynchronize(c->batch->stream));
    c->budget_on = on != 0;
    HIPCHK(c, hipMemsetAsync(c->ws + c->lay.off_budget, 0, 16 * 8, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return CC_OK;
}

cc_status cc_set_clock(cc_ctx* c, double t, int64_t step) {
    if (!c || step < 0 || !std::isfinite(t)) return fail(c, CC_ERR_ARG, "bad argument");
    c->speeds_ready = false;
    c->in_step = false;
    c->t = t;
    c->step = step;
    c->parity = (int)(step & 1);
    cc_status st = levels_at(c, t);
    if (st != CC_OK) return st;
    if (has_body(c)) HIPCHK(c, hipMemsetAsync(c->ws + c->lay.off_stamp, 0xff, c->lay.nc * 4, c->stream));
    return CC_OK;
}

cc_status cc_set_u(cc_ctx* c, const double* d_u) {
    if (!c || !d_u) return fail(c, CC_ERR_ARG, "null argument");
    c->speeds_ready = false;
    size_t n = 4 * c->lay.nc;
    if (fp32(c))
        hipLaunchKernelGGL(k_copy_u<float>, dim3(nblk(n)), dim3(TPB), 0, c->stream, n, d_u,
                           at<float>(c, c->lay.off_u[c->cur]));
    else
        HIPCHK(c, hipMemcpyAsync(at<double>(c, c->lay.off_u[c->cur]), d_u, n * 8, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipGetLastError());
    c->have_state = true;
    return CC_OK;
}

cc_status cc_get_state(cc_ctx* c, double* d_out, int32_t what) {
    if (!c || !d_out || (what != 0 && what != 1)) return fail(c, CC_ERR_ARG, "bad argument");
    size_t n = 4 * c->lay.nc;
    const double* al = c->lev[c->s0].alpha;
    if (what == 1) {
        if (fp32(c))
            hipLaunchKernelGGL(k_u_to_f64<float>, dim3(nblk(n)), dim3(TPB), 0, c->stream, n,
                               at<float>(c, c->lay.off_u[c->cur]), d_out);
        else
            HIPCHK(c, hipMemcpyAsync(d_out, at<double>(c, c->lay.off_u[c->cur]), n * 8, hipMemcpyDeviceToDevice,
                                     c->stream));
    } else {
        if (fp32(c))
            hipLaunchKernelGGL(k_u_to_prim<float>, dim3(nblk(c->lay.nc)), dim3(TPB), 0, c->stream, c->g, al,
                               at<float>(c, c->lay.off_u[c->cur]), d_out);
        else
            hipLaunchKernelGGL(k_u_to_prim<double>, dim3(nblk(c->lay.nc)), dim3(TPB), 0, c->stream, c->g, al,
                               at<double>(c, c->lay.off_u[c->cur]), d_out);
    }
    HIPCHK(c, hipGetLastError());
    return CC_OK;
}

cc_status cc_begin_step(cc_ctx* c, double dt) {
    if (!c) return CC_ERR_ARG;
    cc_status st = not_in_batch(c);
    if (st != CC_OK) return st;
    StepArgs a;
    c->speeds_ready = false;
    if ((st = prepare_step(c, dt, a)) != CC_OK) return st;
    if ((st = own_upload(c, a)) != CC_OK) return st;
    TimedPair tp{};
    tstart(c, 3, tp);
    launch_geometry(c->eng, c->stream);
    tstop(c, tp);
    // the axisymmetric source acts on the level-n state before the first sweep
    if (fp32(c)) launch_axisym<float>(c->eng, c->stream);
    else launch_axisym<double>(c->eng, c->stream);
    HIPCHK(c, hipGetLastError());
    c->in_step = true;
    c->sweeps_done = 0;
    return CC_OK;
}

}  // extern "C"

namespace {

template <typename R>
cc_status own_sweep(cc_ctx* c, int s) {
    Engine& E = c->eng;
    int dir = s == 0 ? c->parity : 1 - c->parity;
    TimedPair tb{};
    tstart(c, 2, tb);
    launch_box_pre<R>(E, c->stream, s);
    tstop(c, tb);
    hipEvent_t ta = nullptr, tz = nullptr;
    if (c->eng.timing & 1) {
        TimedPair tp = engine_pair(c->eng, dir);
        ta = tp.a;
        tz = tp.b;
    }
    launch_dense<R>(E, c->stream, s, 1 << dir, ta, tz);
    tstart(c, 2, tb);
    launch_box_post<R>(E, c->stream, s, 1 << dir);
    tstop(c, tb);
    HIPCHK(c, hipGetLastError());
    return CC_OK;
}

}  // namespace

extern "C" {

cc_status cc_sweep(cc_ctx* c, int32_t dir, double dt) {
    if (!c) return CC_ERR_ARG;
    if (!c->in_step || c->sweeps_done > 1) return fail(c, CC_ERR_ARG, "cc_sweep outside a step");
    int want = c->sweeps_done == 0 ? c->parity : 1 - c->parity;
    if (dir != want) return fail(c, CC_ERR_ARG, "sweep direction out of order");
    if (dt != c->step_dt) return fail(c, CC_ERR_ARG, "dt differs from cc_begin_step");
    int s = c->sweeps_done;
    cc_status st = fp32(c) ? own_sweep<float>(c, s) : own_sweep<double>(c, s);
    if (st != CC_OK) return st;
    c->sweeps_done++;
    c->cur = 1 - c->cur;  // the sweep's output is the current state (both sweeps: unchanged)
    return CC_OK;
}

cc_status cc_end_step(cc_ctx* c) {
    if (!c) return CC_ERR_ARG;
    if (!c->in_step || c->sweeps_done != 2) return fail(c, CC_ERR_ARG, "cc_end_step before both sweeps");
    std::swap(c->s0, c->s1);
    c->t = c->t + c->step_dt;
    c->step++;
    c->parity ^= 1;
    c->in_step = false;
    return CC_OK;
}

}  // extern "C"

namespace {

// Whole step through the context's own captured graph (timed: the same launches one by one,
// the dense launches bracketed by events).
template <typename R>
cc_status own_graph_step(cc_ctx* c, double dt, bool timed = false) {
    Engine& E = c->eng;
    int b = E.buf;
    HIPCHK(c, engine_hostbuf(E, b));
    cc_status st = prepare_step(c, dt, E.h_args[b][0]);
    if (st != CC_OK) return st;
    if (E.extra) std::memcpy(reinterpret_cast<char*>(E.h_args[b]) + sizeof(StepArgs), c->hset.data(), E.extra);
    int dir0 = E.h_args[b][0].sw[0].dir;
    if (timed) {
        step_sequence_timed<R>(E, c->stream, b, dir0);
        HIPCHK(c, hipGetLastError());
    } else {
        HIPCHK(c, engine_graph_step<R>(E, c->stream, b, dir0));
    }
    HIPCHK(c, hipEventRecord(E.ev[b], c->stream));
    E.ev_used[b] = true;
    E.buf = 1 - b;
    c->speeds_ready = true;
    c->speeds_buf = b;
    c->in_step = true;
    c->sweeps_done = 2;
    return CC_OK;
}

}  // namespace

extern "C" {

cc_status cc_step(cc_ctx* c, double dt) {
    if (!c) return CC_ERR_ARG;
    cc_status st = not_in_batch(c);
    if (st != CC_OK) return st;
    if (c->eng.timing & 2) {  // phase timing needs the single sweeps' launches
        if ((st = cc_begin_step(c, dt)) != CC_OK) return st;
        int d1 = c->parity, d2 = 1 - c->parity;
        if ((st = cc_sweep(c, d1, dt)) != CC_OK) return st;
        if ((st = cc_sweep(c, d2, dt)) != CC_OK) return st;
        return cc_end_step(c);
    }
    if (!c->stream) {  // the null stream cannot be captured: individual launches
        if ((st = cc_begin_step(c, dt)) != CC_OK) return st;
        int d1 = c->parity, d2 = 1 - c->parity;
        if ((st = cc_sweep(c, d1, dt)) != CC_OK) return st;
        if ((st = cc_sweep(c, d2, dt)) != CC_OK) return st;
        return cc_end_step(c);
    }
    bool timed = (c->eng.timing & 1) != 0;
    st = fp32(c) ? own_graph_step<float>(c, dt, timed) : own_graph_step<double>(c, dt, timed);
    if (st != CC_OK) return st;
    return cc_end_step(c);
}

}  // extern "C"

namespace {

// Largest speeds |u_x|, |u_y| of the body's vertices at the context's time (0 without a
// body): the wall's part of the CFL condition.
void wall_speeds(cc_ctx* c, double& wsx, double& wsy) {
    wsx = wsy = 0.0;
    for (int b = 0; b < c->nb; b++) {  // several bodies: every body's vertices
        const HostBody& B = c->hb[b];
        std::vector<double> pv(B.verts.size());
        body_pose_xy(c, b, c->t, c->t, pv.data());
        double thd = B.amp * B.omega * std::cos(B.omega * c->t);
        double cx = B.ref_x + B.vx * c->t, cy = B.ref_y + B.vy * c->t;
        for (size_t k = 0; k < pv.size(); k += 2) {
            wsx = std::fmax(wsx, std::fabs(B.vx - thd * (pv[k + 1] - cy)));
            wsy = std::fmax(wsy, std::fabs(B.vy + thd * (pv[k] - cx)));
        }
    }
    if (c->m == 0) return;
    std::vector<double> pv(2 * c->m);
    Pose q = pose_at(c, c->t);
    pose_xy(c, q, q, pv.data());
    double thd = c->amp * c->omega * std::cos(c->omega * c->t);
    double cx = c->ref_x + c->vx * c->t, cy = c->ref_y + c->vy * c->t;
    for (int k = 0; k < c->m; k++) {
        double ux = c->vx - thd * (pv[2 * k + 1] - cy);
        double uy = c->vy + thd * (pv[2 * k] - cx);
        wsx = std::fmax(wsx, std::fabs(ux));
        wsy = std::fmax(wsy, std::fabs(uy));
    }
}

// Wave speeds (bit patterns from the reduction) plus the body's vertex speeds -> dt.
double dt_from_speeds(cc_ctx* c, double cfl, double sx, double sy) {
    double wsx, wsy;
    wall_speeds(c, wsx, wsy);
    sx = std::fmax(sx, wsx);
    sy = std::fmax(sy, wsy);
    return cfl * std::fmin(c->hx / sx, c->hy / sy);
}

// Status bit 1 (a cell turned fluid, or was emptied, with no donor next to it) is reported
// but refuses nothing: such a cell keeps no content, its faces carry nothing, and it takes
// content from the first donor that appears (the oracle runs on the same way).
cc_status status_error(cc_ctx* c, unsigned int status, double sx, double sy) {
    if (status & 2u) return fail(c, CC_ERR_STATE, "a cut cell stayed inadmissible after two collapse rounds");
    if (status & 4u) return fail(c, CC_ERR_UNSUPPORTED, "two bodies meet in one face or cell");
    if (status & 8u) return fail(c, CC_ERR_DEVICE, "a grid barrier of the persistent sweep timed out");
    if (!std::isfinite(sx) || !std::isfinite(sy)) return fail(c, CC_ERR_STATE, "non-finite or non-physical state");
    return CC_OK;
}

}  // namespace

extern "C" {

cc_status cc_cfl_dt(cc_ctx* c, double cfl, double* h_dt, double* d_dt) {
    if (!c || (!h_dt && !d_dt) || !(cfl > 0.0)) return fail(c, CC_ERR_ARG, "bad argument");
    if (c->in_step) return fail(c, CC_ERR_ARG, "cc_cfl_dt inside a step");
    if (d_dt) {  // asynchronous: the reduction and the time step on the device
        unsigned long long* smax = at<unsigned long long>(c, c->lay.off_smax);
        unsigned long long* part = at<unsigned long long>(c, c->lay.off_part);
        const double* al = c->lev[c->s0].alpha;
        int blocks = (int)std::min<size_t>(CFL_MAX_BLOCKS, nblk(c->lay.nc));
        if (fp32(c))
            hipLaunchKernelGGL(k_cfl<float>, dim3(blocks), dim3(256), 0, c->stream, c->g, al,
                               at<float>(c, c->lay.off_u[c->cur]), part);
        else
            hipLaunchKernelGGL(k_cfl<double>, dim3(blocks), dim3(256), 0, c->stream, c->g, al,
                               at<double>(c, c->lay.off_u[c->cur]), part);
        hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(256), 0, c->stream, blocks, (const unsigned long long*)part,
                           smax);
        double wsx, wsy;
        wall_speeds(c, wsx, wsy);
        hipLaunchKernelGGL(k_cfl_dt, dim3(1), dim3(64), 0, c->stream, (const unsigned long long*)smax,
                           (const unsigned int*)at<unsigned int>(c, c->lay.off_status), wsx, wsy, c->hx, c->hy, cfl,
                           d_dt);
        HIPCHK(c, hipGetLastError());
        if (!h_dt) return CC_OK;
    }
    if (c->speeds_ready && !c->batch) {  // reduced and read back by the last captured step
        HIPCHK(c, wait_event(c->eng.ev[c->speeds_buf]));
        double sx, sy;
        std::memcpy(&sx, &c->eng.h_cflout[0], 8);
        std::memcpy(&sy, &c->eng.h_cflout[1], 8);
        cc_status st = status_error(c, c->eng.h_gather[0], sx, sy);
        if (st != CC_OK) return st;
        *h_dt = dt_from_speeds(c, cfl, sx, sy);
        return CC_OK;
    }
    unsigned long long* smax = at<unsigned long long>(c, c->lay.off_smax);
    unsigned long long* part = at<unsigned long long>(c, c->lay.off_part);
    const double* al = c->lev[c->s0].alpha;
    int blocks = (int)std::min<size_t>(CFL_MAX_BLOCKS, nblk(c->lay.nc));
    if (fp32(c))
        hipLaunchKernelGGL(k_cfl<float>, dim3(blocks), dim3(256), 0, c->stream, c->g, al,
                           at<float>(c, c->lay.off_u[c->cur]), part);
    else
        hipLaunchKernelGGL(k_cfl<double>, dim3(blocks), dim3(256), 0, c->stream, c->g, al,
                           at<double>(c, c->lay.off_u[c->cur]), part);
    hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(256), 0, c->stream, blocks, (const unsigned long long*)part, smax);
    HIPCHK(c, hipGetLastError());
    // one read-back: the two maxima and the status word are adjacent
    unsigned long long hs[3];
    HIPCHK(c, hipMemcpyAsync(hs, smax, 16, hipMemcpyDeviceToHost, c->stream));
    unsigned int status = 0;
    HIPCHK(c, hipMemcpyAsync(&status, c->ws + c->lay.off_status, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double sx, sy;
    std::memcpy(&sx, &hs[0], 8);
    std::memcpy(&sy, &hs[1], 8);
    cc_status st = status_error(c, status, sx, sy);
    if (st != CC_OK) return st;
    *h_dt = dt_from_speeds(c, cfl, sx, sy);
    return CC_OK;
}

}  // extern "C"

namespace {

void plan_const(cc_ctx* c, double cfl, PlanConst& P) {
    std::memset(&P, 0, sizeof(P));
    base_args(c, P.base);
    P.base.pc = at<PlanConst>(c, c->lay.off_pconst);
    P.base.ps = at<PlanState>(c, c->lay.off_pstate);
    P.base.dtlog = at<double>(c, c->lay.off_dtlog);
    P.body = at<double>(c, c->lay.off_body);
    P.m = c->m;
    P.ref_x = c->ref_x;
    P.ref_y = c->ref_y;
    P.theta0 = c->theta0;
    P.vx = c->vx;
    P.vy = c->vy;
    P.amp = c->amp;
    P.omega = c->omega;
    P.cs0 = std::cos(c->theta0);
    P.sn0 = std::sin(c->theta0);
    P.cert0 = c->cert0;
    P.ext0 = c->ext0;
    P.x_lo = c->cfg.x_lo;
    P.x_hi = c->cfg.x_hi;
    P.y_lo = c->cfg.y_lo;
    P.y_hi = c->cfg.y_hi;
    P.hx = c->hx;
    P.hy = c->hy;
    P.nx = c->g.nx;
    P.ny = c->g.ny;
    P.gw = c->lay.gw;
    P.gh = c->lay.gh;
    P.capw = c->lay.capw;
    P.caph = c->lay.caph;
    P.u[0] = c->ws + c->lay.off_u[0];
    P.u[1] = c->ws + c->lay.off_u[1];
    P.cfl = cfl;
}

void plan_state_from(const cc_ctx* c, PlanState& S) {
    std::memset(&S, 0, sizeof(S));
    S.t = c->t;
    S.step_dt = c->step_dt;
    S.step = c->step;
    S.parity = c->parity;
    S.s0 = c->s0;
    S.sm = c->sm;
    S.s1 = c->s1;
    S.cur = c->cur;
    for (int k = 0; k < 3; k++) {
        S.lbox[k] = c->lbox[k];
        S.lev[k] = c->lev[k];
    }
    S.mot = c->mot;
    S.last_sweep_box = c->last_sweep_box;
}

void plan_state_to(cc_ctx* c, const PlanState& S) {
    c->t = S.t;
    c->step_dt = S.step_dt;
    c->step = S.step;
    c->parity = S.parity;
    c->s0 = S.s0;
    c->s1 = S.s1;
    for (int k = 0; k < 3; k++) {
        c->lbox[k] = S.lbox[k];
        c->lev[k].poly = S.lev[k].poly;
    }
    c->mot = S.mot;
    c->last_sweep_box = S.last_sweep_box;
}

// speeds: where the run kept the context's wave-speed maxima.
cc_status halt_error(cc_ctx* c, int halt, const unsigned long long* speeds) {
    switch (halt) {
        case HALT_STATUS:
        case HALT_SPEEDS: {
            unsigned long long sp[2];
            unsigned int st = 0;
            HIPCHK(c, hipMemcpyAsync(sp, speeds, 16, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipMemcpyAsync(&st, at<unsigned int>(c, c->lay.off_status), 4, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            double sx, sy;
            std::memcpy(&sx, &sp[0], 8);
            std::memcpy(&sy, &sp[1], 8);
            cc_status e = status_error(c, st, sx, sy);
            return e != CC_OK ? e : fail(c, CC_ERR_STATE, "non-finite or non-physical state");
        }
        case HALT_DT: return fail(c, CC_ERR_MOTION, "dt must be positive");
        case HALT_MOTION: return fail(c, CC_ERR_MOTION, "the body moves a cell or more within one sweep");
        case HALT_REGION: return fail(c, CC_ERR_WORKSPACE, "geometry region exceeds capacity");
        default: return fail(c, CC_ERR_WORKSPACE, "sweep region exceeds the staging capacity");
    }
}

// Device-planned steps of every member of engine E (a context's own engine: one member):
// member k's arguments at E.d_args + k, its speed maxima at E.d_cflout + 2k.  h_dt: member
// k's time steps at h_dt[k nsteps ...]; done[k]: its completed steps; bad: the first member
// that stopped early (-1: none), whose error the return value and its message give.
template <typename R>
cc_status advance_members(Engine& E, hipStream_t s, int nsteps, double cfl, double* h_dt, float* h_step_ms,
                          std::vector<int>& done, int& bad) {
    int n = (int)E.mem.size();
    bool single = n == 1 && E.cap_n == 1;
    cc_ctx* c0 = E.mem[0];
    done.assign(n, 0);
    bad = -1;
    auto dev_fail = [&](hipError_t e) {
        return fail(c0, CC_ERR_DEVICE, std::string("device-planned steps: ") + hipGetErrorString(e));
    };
    hipError_t e = hipStreamSynchronize(s);
    for (int k = 0; k < n && e == hipSuccess; k++) {
        cc_ctx* c = E.mem[k];
        PlanConst P;
        plan_const(c, cfl, P);
        P.base.cfl_out = E.d_cflout + 2 * k;
        e = hipMemcpy(at<PlanConst>(c, c->lay.off_pconst), &P, sizeof(P), hipMemcpyHostToDevice);
        // wave speeds of the start state: the first step's CFL condition
        unsigned long long* part = at<unsigned long long>(c, c->lay.off_part);
        int blocks = (int)std::min<size_t>(CFL_MAX_BLOCKS, nblk(c->lay.nc));
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_cfl<R>, dim3(blocks), dim3(256), 0, s, c->g, c->lev[c->s0].alpha,
                               at<R>(c, c->lay.off_u[c->cur]), part);
            hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(256), 0, s, blocks, (const unsigned long long*)part,
                               E.d_cflout + 2 * k);
            e = hipGetLastError();
        }
    }
    if (e != hipSuccess) return dev_fail(e);
    std::vector<hipEvent_t> ev;
    auto drop_events = [&]() {
        for (auto& x : ev)
            if (x) (void)hipEventDestroy(x);
    };
    if (h_step_ms) {
        ev.assign((size_t)nsteps + 1, nullptr);
        for (auto& x : ev)
            if ((e = hipEventCreate(&x)) != hipSuccess) break;
        if (e != hipSuccess) {
            drop_events();
            return dev_fail(e);
        }
    }
    int base = 0;
    bool running = true;
    std::vector<int> halted(n, 0);
    while (base < nsteps && running) {
        int m = std::min(nsteps - base, DTLOG);
        std::vector<PlanState> S(n);
        for (int k = 0; k < n && e == hipSuccess; k++) {
            plan_state_from(E.mem[k], S[k]);
            S[k].remaining = m;
            S[k].halt = halted[k];  // a member that stopped stays stopped
            e = hipMemcpy(at<PlanState>(E.mem[k], E.mem[k]->lay.off_pstate), &S[k], sizeof(PlanState),
                          hipMemcpyHostToDevice);
        }
        if (!ev.empty() && e == hipSuccess) e = hipEventRecord(ev[base], s);
        // the run's first step of each member is planned by a launch of its own, every later
        // one by the last block of the step before it
        for (int k = 0; k < n && e == hipSuccess; k++) {
            cc_ctx* c = E.mem[k];
            hipLaunchKernelGGL(kb_plan, dim3(1), dim3(T_PLAN), 0, s, (const PlanConst*)at<PlanConst>(c, c->lay.off_pconst),
                               at<PlanState>(c, c->lay.off_pstate), E.d_args + k, at<double>(c, c->lay.off_dtlog));
            e = hipGetLastError();
        }
        for (int i = 0; i < m && e == hipSuccess;) {
            // runs of steps in one graph unless every step is timed on its own
            int k = ev.empty() && m - i >= PLANNED_RUN ? PLANNED_RUN : 1;
            e = engine_planned_step<R>(E, s, single ? (c0->parity + i) & 1 : -1, k);
            if (!ev.empty() && e == hipSuccess) e = hipEventRecord(ev[base + i + 1], s);
            i += k;
        }
        std::vector<double> dts((size_t)n * m);
        for (int k = 0; k < n && e == hipSuccess; k++) {
            cc_ctx* c = E.mem[k];
            e = hipMemcpyAsync(&S[k], at<PlanState>(c, c->lay.off_pstate), sizeof(PlanState), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(dts.data() + (size_t)k * m, at<double>(c, c->lay.off_dtlog), (size_t)m * 8,
                                   hipMemcpyDeviceToHost, s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            drop_events();
            return dev_fail(e);
        }
        running = false;
        for (int k = 0; k < n; k++) {
            cc_ctx* c = E.mem[k];
            plan_state_to(c, S[k]);
            if (h_dt)
                std::copy(dts.begin() + (size_t)k * m, dts.begin() + (size_t)k * m + S[k].steps,
                          h_dt + (size_t)k * nsteps + done[k]);
            done[k] += S[k].steps;
            halted[k] = S[k].halt;
            if (S[k].halt) {
                if (bad < 0) bad = k;
            } else {
                running = true;
            }
        }
        if (h_step_ms)
            for (int i = 0; i < m; i++)
                if (hipEventElapsedTime(&h_step_ms[base + i], ev[base + i], ev[base + i + 1]) != hipSuccess)
                    h_step_ms[base + i] = -1.0f;
        base += m;
    }
    drop_events();
    for (cc_ctx* c : E.mem) c->speeds_ready = false;
    if (bad < 0) return CC_OK;
    return halt_error(E.mem[bad], halted[bad], E.d_cflout + 2 * bad);
}

template <typename R>
cc_status advance(cc_ctx* c, int nsteps, double cfl, double* h_dt, float* h_step_ms) {
    std::vector<int> done;
    int bad = -1;
    cc_status st = advance_members<R>(c->eng, c->stream, nsteps, cfl, h_dt, h_step_ms, done, bad);
    c->advanced = done.empty() ? 0 : done[0];
    return st;
}

template <typename R>
cc_status batch_advance(cc_batch* b, int nsteps, double cfl, double* h_dt, float* h_step_ms, int32_t* h_done) {
    Engine& E = b->eng;
    std::vector<int> done;
    int bad = -1;
    cc_status st = advance_members<R>(E, b->stream, nsteps, cfl, h_dt, h_step_ms, done, bad);
    if (h_done)
        for (size_t k = 0; k < done.size(); k++) h_done[k] = done[k];
    if (st != CC_OK) {
        int k = bad >= 0 ? bad : 0;
        b->err = "member " + std::to_string(k) + ": " + E.mem[k]->err;
    }
    return st;
}

}  // namespace

extern "C" {

cc_status cc_advance(cc_ctx* c, int32_t nsteps, double cfl, double* h_dt, float* h_step_ms, int32_t* h_done) {
    if (!c) return CC_ERR_ARG;
    cc_status st = not_in_batch(c);
    if (st != CC_OK) return st;
    if (h_done) *h_done = 0;
    if (c->nb > 1) return fail(c, CC_ERR_UNSUPPORTED, "several bodies: steps are planned on the host (cc_step)");
    if (c->eng.axisym) return fail(c, CC_ERR_UNSUPPORTED, "axisymmetric form: steps are planned on the host (cc_step)");
    if (nsteps < 0 || !(cfl > 0.0) || !std::isfinite(cfl)) return fail(c, CC_ERR_ARG, "bad argument");
    if (c->in_step) return fail(c, CC_ERR_ARG, "cc_advance inside a step");
    if (!c->have_state) return fail(c, CC_ERR_ARG, "no state set");
    if (nsteps == 0) return CC_OK;
    c->advanced = 0;
    st = fp32(c) ? advance<float>(c, nsteps, cfl, h_dt, h_step_ms) : advance<double>(c, nsteps, cfl, h_dt, h_step_ms);
    if (h_done) *h_done = c->advanced;
    return st;
}

cc_status cc_totals(cc_ctx* c, double* h_totals4, double* h_budget12) {
    if (!c || !h_totals4) return fail(c, CC_ERR_ARG, "bad argument");
    if (h_budget12) {
        if (c->batch) HIPCHK(c, hipStreamSynchronize(c->batch->stream));
        HIPCHK(c, hipMemcpyAsync(h_budget12, c->ws + c->lay.off_budget, 12 * 8, hipMemcpyDeviceToHost, c->stream));
    }
    size_t nc = c->lay.nc;
    size_t chunk = (nc + NPART - 1) / NPART;
    double* part = at<double>(c, c->lay.off_part);
    double* tot = at<double>(c, c->lay.off_tot);
    if (fp32(c))
        hipLaunchKernelGGL(k_sum_partial<float>, dim3(NPART, 4), dim3(RT), 0, c->stream, nc, 4,
                           at<float>(c, c->lay.off_u[c->cur]), chunk, part);
    else
        hipLaunchKernelGGL(k_sum_partial<double>, dim3(NPART, 4), dim3(RT), 0, c->stream, nc, 4,
                           at<double>(c, c->lay.off_u[c->cur]), chunk, part);
    hipLaunchKernelGGL(k_sum_final, dim3(4), dim3(RT), 0, c->stream, NPART, (const double*)part, 1.0, tot);
    HIPCHK(c, hipGetLastError());
    double h[4];
    HIPCHK(c, hipMemcpyAsync(h, tot, 32, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double area = c->hx * c->hy;
    for (int k = 0; k < 4; k++) h_totals4[k] = h[k] * area;
    return CC_OK;
}

}  // extern "C"

// Scratch of cc_totals_state: the per-block partial sums (4 components x NPART blocks) of
// the deterministic sum.  Every device the library runs on holds its own copy until the
// process ends.  Host code must not use this name as a device address (on the host it is
// only a stand-in for the symbol); it uses the address hipGetSymbolAddress returns for
// the current device.
static __device__ __align__(256) double scratch[4 * NPART];

namespace {

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[SCRATCH_DEVICES] = {};

// Device address of the current device's scratch array, looked up on the first call on
// that device (with the device current) and kept.
hipError_t scratch_address(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= SCRATCH_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

cc_status cc_totals_state(const void* d_u, int32_t precision, int32_t nx, int32_t ny, double hx, double hy,
                          void* hip_stream, double* d_out4) {
    auto bad = [](cc_status st, const char* msg) {
        g_create_err = msg;
        return st;
    };
    if (!d_u || !d_out4 || nx < 1 || ny < 1 || (precision != CC_FP64 && precision != CC_FP32_GEOM64) ||
        !std::isfinite(hx) || !std::isfinite(hy))
        return bad(CC_ERR_ARG, "bad argument");
    size_t nc = (size_t)nx * (size_t)ny;
    if (nc > (size_t)CC_TOTALS_STATE_MAX_CELLS)
        return bad(CC_ERR_UNSUPPORTED, "state larger than CC_TOTALS_STATE_MAX_CELLS cells");
    double* part = nullptr;
    hipError_t e = scratch_address(&part);
    if (e != hipSuccess) return bad(CC_ERR_DEVICE, "scratch address lookup failed");
    hipStream_t s = (hipStream_t)hip_stream;
    size_t chunk = (nc + NPART - 1) / NPART;
    // the same launches as cc_totals, so the two agree bit for bit
    if (precision == CC_FP32_GEOM64)
        hipLaunchKernelGGL(k_sum_partial<float>, dim3(NPART, 4), dim3(RT), 0, s, nc, 4, (const float*)d_u, chunk,
                           part);
    else
        hipLaunchKernelGGL(k_sum_partial<double>, dim3(NPART, 4), dim3(RT), 0, s, nc, 4, (const double*)d_u, chunk,
                           part);
    hipLaunchKernelGGL(k_sum_final, dim3(4), dim3(RT), 0, s, NPART, (const double*)part, hx * hy, d_out4);
    if (hipGetLastError() != hipSuccess) return bad(CC_ERR_DEVICE, "launch failed");
    return CC_OK;
}

}  // extern "C"

namespace {

// The gas's velocity field of the bodies at the context's time, for the loads kernels.
void loads_bodies(const cc_ctx* c, LoadsArgs& a) {
    std::memset(a.bv, 0, sizeof(a.bv));
    if (c->nb > 1) {
        for (int b = 0; b < c->nb; b++) {
            const HostBody& B = c->hb[b];
            a.bv[b] = BodyVel{B.vx, B.vy, B.amp * B.omega * std::cos(B.omega * c->t), B.ref_x + B.vx * c->t,
                              B.ref_y + B.vy * c->t};
        }
        return;
    }
    a.bv[0] = BodyVel{c->vx, c->vy, c->amp * c->omega * std::cos(c->omega * c->t), c->ref_x + c->vx * c->t,
                      c->ref_y + c->vy * c->t};
}

cc_status loads_of(cc_ctx* c, int body, double* h_out4) {
    if (!c || !h_out4) return fail(c, CC_ERR_ARG, "bad argument");
    if (c->in_step) return fail(c, CC_ERR_ARG, "surface loads inside a step");
    if (!c->have_state) return fail(c, CC_ERR_ARG, "no state set");
    if (body < 0 || body >= std::max(c->nb, 1)) return fail(c, CC_ERR_ARG, "no such body");
    for (int k = 0; k < 4; k++) h_out4[k] = 0.0;
    const Box& reg = c->lbox[c->s0];
    if (!has_body(c) || box_empty(reg)) return CC_OK;
    LoadsArgs a;
    a.g = c->g;
    a.L = c->lev[c->s0];
    a.reg = reg;
    loads_bodies(c, a);
    a.body = body;
    int blocks = (int)std::min<size_t>(LOADS_MAX_BLOCKS, nblk((size_t)reg.w() * reg.h(), LOADS_T));
    double* part = at<double>(c, c->lay.off_part);
    double* out = at<double>(c, c->lay.off_tot);
    if (fp32(c))
        hipLaunchKernelGGL(k_loads<float>, dim3(blocks), dim3(LOADS_T), 0, c->stream, a,
                           (const float*)at<float>(c, c->lay.off_u[c->cur]), part);
    else
        hipLaunchKernelGGL(k_loads<double>, dim3(blocks), dim3(LOADS_T), 0, c->stream, a,
                           (const double*)at<double>(c, c->lay.off_u[c->cur]), part);
    hipLaunchKernelGGL(k_loads_final, dim3(1), dim3(64), 0, c->stream, blocks, (const double*)part, out);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(h_out4, out, 32, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return CC_OK;
}

}  // namespace

extern "C" {

cc_status cc_surface_loads(cc_ctx* c, double* h_out4) {
    if (c && c->nb > 1) return fail(c, CC_ERR_UNSUPPORTED, "several bodies: the loads of each (cc_body_loads)");
    return loads_of(c, 0, h_out4);
}

cc_status cc_body_loads(cc_ctx* c, int32_t body, double* h_out4) { return loads_of(c, body, h_out4); }

cc_status cc_surface_pressure(cc_ctx* c, double* d_out, int32_t max_records, int32_t* h_n) {
    if (!c || !h_n || max_records < 0 || (max_records > 0 && !d_out)) return fail(c, CC_ERR_ARG, "bad argument");
    if (c->in_step) return fail(c, CC_ERR_ARG, "cc_surface_pressure inside a step");
    if (!c->have_state) return fail(c, CC_ERR_ARG, "no state set");
    *h_n = 0;
    const Box& R = c->lbox[c->s0];
    if (!has_body(c) || box_empty(R)) return CC_OK;
    LoadsArgs a;
    a.g = c->g;
    a.L = c->lev[c->s0];
    a.reg = R;
    loads_bodies(c, a);
    a.body = 0;
    int cells = R.w() * R.h();
    int chunk = (cells + CUT_BLOCKS - 1) / CUT_BLOCKS, nb = (cells + chunk - 1) / chunk;
    int* counts = at<int>(c, c->lay.off_part);  // 4 KiB of the reduction scratch
    int* total = at<int>(c, c->lay.off_tot);
    // the list of wall cells (at most the region's cells) in the box staging, unused
    // outside a step: 4 B per cell against its 32 B per capacity cell
    int* list = at<int>(c, c->lay.off_sQ);
    auto run = [&](auto* U) {
        using R_ = std::remove_const_t<std::remove_pointer_t<decltype(U)>>;
        WallCells<R_> pred{c->g, a.L, U};
        hipLaunchKernelGGL(k_list_count<WallCells<R_>>, dim3(nb), dim3(CUT_T), 0, c->stream, pred, R, chunk, counts);
        hipLaunchKernelGGL(k_cut_scan, dim3(1), dim3(CUT_T), 0, c->stream, nb, counts, total);
        hipLaunchKernelGGL(k_list_write<WallCells<R_>>, dim3(nb), dim3(CUT_T), 0, c->stream, pred, R, chunk,
                           (const int*)counts, list);
        if (max_records > 0)
            hipLaunchKernelGGL(k_wall_records<R_>, dim3(nblk((size_t)max_records, LOADS_T)), dim3(LOADS_T), 0,
                               c->stream, a, U, (const int*)list, (const int*)total, (int)max_records, d_out);
    };
    if (fp32(c)) run((const float*)at<float>(c, c->lay.off_u[c->cur]));
    else run((const double*)at<double>(c, c->lay.off_u[c->cur]));
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(h_n, total, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return CC_OK;
}

cc_status cc_info(cc_ctx* c, double* h_out, int32_t n) {
    if (!c || !h_out || n < 1) return fail(c, CC_ERR_ARG, "bad argument");
    unsigned int dev[2];
    HIPCHK(c, hipMemcpyAsync(&dev[0], c->ws + c->lay.off_status, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&dev[1], c->ws + c->lay.off_ncol, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double v[11] = {c->t, (double)c->step, (double)c->parity, (double)dev[0], (double)dev[1],
                    (double)c->last_sweep_box.w() * c->last_sweep_box.h(), (double)c->lay.cap,
                    (double)X_RB[c->eng.tile_x], (double)Y_TR[c->eng.tile_y], y_walk(c->eng.tile_y) ? 1.0 : 0.0,
                    c->eng.merge_x ? 1.0 : 0.0};
    for (int k = 0; k < n && k < 11; k++) h_out[k] = v[k];
    return CC_OK;
}

}  // extern "C"

namespace {

// Tuning arguments of a context: both sweeps over the whole grid (no box), from the current
// state into the spare state buffer, which the next sweep overwrites.
void tune_args(cc_ctx* c, StepArgs& a) {
    base_args(c, a);
    for (int s = 0; s < 2; s++) {
        SweepJob& J = a.sw[s];
        J.B = Box{0, 0, 0, 0};
        J.dir = s;
        J.lam = 0.25 * std::min(c->hx, c->hy) / std::max(c->hx, c->hy);
        J.Uin = c->ws + c->lay.off_u[c->cur];
        J.Uout = c->ws + c->lay.off_u[1 - c->cur];
    }
}

// Times every valid tile variant of both dense sweeps for the members of engine E (their
// tuning arguments already in device memory), reps launches each, as a step launches them
// (beside the first box phase, whose idle blocks set the launch's occupancy), and keeps
// the fastest: the current variant unless another is at least 3 % faster, so that timing
// noise between near-equal shapes does not flip the choice.  The launch plan is rebuilt
// for every variant, which destroys the captured step graphs: the caller has drained the
// stream.  err: set on failure.
template <typename R>
bool tune_engine(Engine& E, hipStream_t s, int reps, std::string& err) {
    hipEvent_t ea, eb;
    if (hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess) {
        err = "event create";
        return false;
    }
    bool ok = true;
    int keep[2] = {E.tile_x, E.tile_y};
    for (int dir = 0; dir < 2 && ok; dir++) {
        int nv = dir == 0 ? NX_VARIANTS : NY_VARIANTS, best = -1;
        float best_ms = 0.0f;
        for (int i = -1; i < nv; i++) {
            int v = i < 0 ? keep[dir] : i;
            if ((i >= 0 && v == keep[dir]) || !dense_variant_ok(E.prec, dir, v)) continue;
            (dir == 0 ? E.tile_x : E.tile_y) = v;
            if (engine_plan(E, s) != hipSuccess) {
                err = "tile plan";
                ok = false;
                break;
            }
            launch_dense<R>(E, s, dir, 1 << dir, nullptr, nullptr, 0, dir == 1 || E.merge_x);  // warm-up
            float ms = 0.0f;
            if (hipEventRecord(ea, s) != hipSuccess) {
                err = "event record";
                ok = false;
                break;
            }
            for (int r = 0; r < reps; r++)
                launch_dense<R>(E, s, dir, 1 << dir, nullptr, nullptr, 0, dir == 1 || E.merge_x);
            if (hipEventRecord(eb, s) != hipSuccess || hipEventSynchronize(eb) != hipSuccess ||
                hipEventElapsedTime(&ms, ea, eb) != hipSuccess || hipGetLastError() != hipSuccess) {
                err = "tile timing failed";
                ok = false;
                break;
            }
            if (best < 0 || ms < 0.97f * best_ms) {
                best = v;
                best_ms = ms;
            }
        }
        keep[dir] = best >= 0 ? best : keep[dir];
        (dir == 0 ? E.tile_x : E.tile_y) = keep[dir];
    }
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
    if (engine_plan(E, s) != hipSuccess && ok) {
        err = "tile plan";
        ok = false;
    }
    return ok;
}

// Tile-choice cache: one line per tuned configuration, "key tile_x tile_y", the key naming
// the device, the precision and the members' grids (a batch's in membership order).
std::string tune_key(int prec, const std::vector<cc_ctx*>& mem) {
    hipDeviceProp_t prop;
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    for (auto& ch : arch)
        if (ch == ' ' || ch == ':') ch = '_';
    std::string k = arch + "/p" + std::to_string(prec);
    for (const cc_ctx* c : mem) k += "/" + std::to_string(c->g.nx) + "x" + std::to_string(c->g.ny);
    return k;
}

bool tune_cache_read(const char* path, const std::string& key, int prec, int& tx, int& ty) {
    if (!path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char kbuf[4096];
    int a = 0, b = 0;
    bool found = false;
    while (std::fscanf(f, "%4095s %d %d", kbuf, &a, &b) == 3)
        if (key == kbuf && dense_variant_ok(prec, 0, a) && dense_variant_ok(prec, 1, b)) {
            tx = a;
            ty = b;
            found = true;  // the last entry for the key wins
        }
    std::fclose(f);
    return found;
}

void tune_cache_write(const char* path, const std::string& key, int tx, int ty) {
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d\n", key.c_str(), tx, ty);
    std::fclose(f);
}

}  // namespace

extern "C" {

cc_status cc_autotune(cc_ctx* c, int32_t reps, int32_t* h_choice, const char* cache_path) {
    if (!c || reps < 1) return fail(c, CC_ERR_ARG, "bad argument");
    if (c->in_step || !c->have_state) return fail(c, CC_ERR_ARG, "cc_autotune needs a state and no open step");
    cc_status st = not_in_batch(c);
    if (st != CC_OK) return st;
    if (c->nb > 1) return fail(c, CC_ERR_UNSUPPORTED, "several bodies: the default tiles");
    Engine& E = c->eng;
    std::string key = tune_key(E.prec, E.mem);
    int tx = 0, ty = 0;
    HIPCHK(c, hipStreamSynchronize(c->stream));  // the captured graphs are about to be destroyed
    if (tune_cache_read(cache_path, key, E.prec, tx, ty)) {
        E.tile_x = tx;
        E.tile_y = ty;
        HIPCHK(c, engine_plan(E, c->stream));
    } else {
        StepArgs a;
        tune_args(c, a);
        if ((st = own_upload(c, a)) != CC_OK) return st;
        std::string err;
        bool ok = fp32(c) ? tune_engine<float>(E, c->stream, reps, err) : tune_engine<double>(E, c->stream, reps, err);
        if (!ok) return fail(c, CC_ERR_DEVICE, err);
        tune_cache_write(cache_path, key, E.tile_x, E.tile_y);
    }
    if (h_choice) {
        h_choice[0] = E.tile_x;
        h_choice[1] = E.tile_y;
    }
    return CC_OK;
}

cc_status cc_batch_autotune(cc_batch* b, int32_t reps, int32_t* h_choice, const char* cache_path) {
    if (!b || reps < 1) return CC_ERR_ARG;
    Engine& E = b->eng;
    int n = (int)E.mem.size();
    if (n == 0) return bfail(b, CC_ERR_ARG, "cc_batch_autotune needs members");
    std::string key = tune_key(E.prec, E.mem);
    int tx = 0, ty = 0;
    BHIPCHK(b, hipStreamSynchronize(b->stream));  // the captured graphs are about to be destroyed
    if (tune_cache_read(cache_path, key, E.prec, tx, ty)) {
        E.tile_x = tx;
        E.tile_y = ty;
        BHIPCHK(b, engine_plan(E, b->stream));
    } else {
        int buf = E.buf;
        BHIPCHK(b, engine_hostbuf(E, buf));
        for (int k = 0; k < n; k++) tune_args(E.mem[k], E.h_args[buf][k]);
        BHIPCHK(b, engine_upload(E, b->stream, buf));
        BHIPCHK(b, hipStreamSynchronize(b->stream));
        std::string err;
        bool ok = E.prec == CC_FP32_GEOM64 ? tune_engine<float>(E, b->stream, reps, err)
                                           : tune_engine<double>(E, b->stream, reps, err);
        if (!ok) return bfail(b, CC_ERR_DEVICE, err);
        tune_cache_write(cache_path, key, E.tile_x, E.tile_y);
    }
    if (h_choice) {
        h_choice[0] = E.tile_x;
        h_choice[1] = E.tile_y;
    }
    return CC_OK;
}

cc_status cc_set_launch_mode(cc_ctx* c, int32_t mode) {
    if (!c) return CC_ERR_ARG;
    if (mode != CC_LAUNCH_PER_PHASE && mode != CC_LAUNCH_PERSISTENT) return fail(c, CC_ERR_ARG, "unknown launch mode");
    if (c->in_step) return fail(c, CC_ERR_ARG, "cc_set_launch_mode inside a step");
    if (mode == CC_LAUNCH_PERSISTENT && (c->nb > 1 || c->eng.axisym))
        return fail(c, CC_ERR_UNSUPPORTED, "several bodies or axisymmetric form: one launch per phase");
    if (mode == CC_LAUNCH_PERSISTENT && c->budget_on)
        return fail(c, CC_ERR_UNSUPPORTED, "the budget is not tracked in the persistent launch mode");
    HIPCHK(c, hipStreamSynchronize(c->stream));  // the captured graphs are about to be destroyed
    c->eng.mode = mode;
    HIPCHK(c, engine_plan(c->eng, c->stream));
    return CC_OK;
}

cc_status cc_set_tiles(cc_ctx* c, int32_t tile_x, int32_t tile_y) {
    if (!c) return CC_ERR_ARG;
    if (!dense_variant_ok(c->eng.prec, 0, tile_x) || !dense_variant_ok(c->eng.prec, 1, tile_y))
        return fail(c, CC_ERR_ARG, "tile variant out of range for this precision");
    if (c->in_step) return fail(c, CC_ERR_ARG, "cc_set_tiles inside a step");
    HIPCHK(c, hipStreamSynchronize(c->stream));  // the captured graphs are about to be destroyed
    c->eng.tile_x = tile_x;
    c->eng.tile_y = tile_y;
    HIPCHK(c, engine_plan(c->eng, c->stream));
    return CC_OK;
}

cc_status cc_timing(cc_ctx* c, int32_t enable) {
    if (!c) return CC_ERR_ARG;
    c->eng.timing = enable & 3;
    return CC_OK;
}

cc_status cc_timing_read(cc_ctx* c, double* h_out, int32_t n) {
    if (!c || !h_out) return fail(c, CC_ERR_ARG, "bad argument");
    HIPCHK(c, engine_timing_read(c->eng, c->stream, h_out, n));
    return CC_OK;
}

cc_status cc_batch_timing(cc_batch* b, int32_t enable) {
    if (!b) return CC_ERR_ARG;
    b->eng.timing = enable & 1;
    return CC_OK;
}

cc_status cc_batch_timing_read(cc_batch* b, double* h_out, int32_t n) {
    if (!b || !h_out) return CC_ERR_ARG;
    BHIPCHK(b, engine_timing_read(b->eng, b->stream, h_out, n));
    return CC_OK;
}

// ------------------------------------------------------------------------------ batches

size_t cc_batch_workspace_bytes(int32_t max_instances) {
    if (max_instances < 1) return 0;
    size_t n = (size_t)max_instances;
    return up(n * sizeof(StepArgs)) + up((size_t)NKINDS * (2 * n + 1) * sizeof(int)) + up(24 * n) +
           up(sizeof(GridSync));
}

cc_status cc_batch_create(int32_t max_instances, int32_t precision, void* d_ws, size_t ws_bytes, void* hip_stream,
                          cc_batch** out) {
    if (!out || max_instances < 1 || (precision != CC_FP64 && precision != CC_FP32_GEOM64)) return CC_ERR_ARG;
    *out = nullptr;
    size_t need = cc_batch_workspace_bytes(max_instances);
    if (!d_ws || ws_bytes < need || ((uintptr_t)d_ws % ALIGN) != 0) return CC_ERR_WORKSPACE;
    cc_batch* b = new cc_batch();
    b->stream = (hipStream_t)hip_stream;
    b->ws = (char*)d_ws;
    Engine& E = b->eng;
    E.prec = precision;
    E.cap_n = max_instances;
    size_t n = (size_t)max_instances, o = 0;
    E.d_args = (StepArgs*)(b->ws + o);
    o += up(n * sizeof(StepArgs));
    E.d_off = (int*)(b->ws + o);
    o += up((size_t)NKINDS * (2 * n + 1) * sizeof(int));
    E.d_cflout = (unsigned long long*)(b->ws + o);
    E.d_gather = (unsigned int*)(E.d_cflout + 2 * n);
    o += up(24 * n);
    E.d_sync = (GridSync*)(b->ws + o);
    E.tile_x = 0;
    E.tile_y = 0;
    if (engine_alloc_host(E) != hipSuccess || hipMemsetAsync(E.d_sync, 0, sizeof(GridSync), b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
        engine_free(E);
        delete b;
        return CC_ERR_DEVICE;
    }
    *out = b;
    return CC_OK;
}

cc_status cc_batch_destroy(cc_batch* b) {
    if (!b) return CC_ERR_ARG;
    (void)hipStreamSynchronize(b->stream);
    for (cc_ctx* c : b->eng.mem) c->batch = nullptr;
    engine_free(b->eng);
    delete b;
    return CC_OK;
}

cc_status cc_batch_add(cc_batch* b, cc_ctx* c) {
    if (!b || !c) return CC_ERR_ARG;
    Engine& E = b->eng;
    if (c->batch) return bfail(b, CC_ERR_ARG, "context already in a batch");
    if (c->nb > 1 || c->eng.axisym)
        return bfail(b, CC_ERR_UNSUPPORTED, "a context with several bodies or in axisymmetric form steps on its own");
    if (c->cfg.precision != E.prec) return bfail(b, CC_ERR_ARG, "precision differs from the batch's");
    if ((int)E.mem.size() >= E.cap_n) return bfail(b, CC_ERR_WORKSPACE, "batch is full");
    if (!c->have_state || c->in_step) return bfail(b, CC_ERR_ARG, "context needs a state and no open step");
    if (c->budget_on && E.mode == CC_LAUNCH_PERSISTENT)
        return bfail(b, CC_ERR_UNSUPPORTED, "the context tracks its budget (not in the persistent mode)");
    BHIPCHK(b, hipStreamSynchronize(c->stream));
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    E.mem.push_back(c);
    c->batch = b;
    BHIPCHK(b, engine_plan(E, b->stream));
    return CC_OK;
}

cc_status cc_batch_remove(cc_batch* b, cc_ctx* c) {
    if (!b || !c) return CC_ERR_ARG;
    Engine& E = b->eng;
    auto it = std::find(E.mem.begin(), E.mem.end(), c);
    if (it == E.mem.end()) return bfail(b, CC_ERR_ARG, "context not in this batch");
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    E.mem.erase(it);
    c->batch = nullptr;
    BHIPCHK(b, engine_plan(E, b->stream));
    return CC_OK;
}

cc_status cc_batch_set_tiles(cc_batch* b, int32_t tile_x, int32_t tile_y) {
    if (!b) return CC_ERR_ARG;
    if (!dense_variant_ok(b->eng.prec, 0, tile_x) || !dense_variant_ok(b->eng.prec, 1, tile_y))
        return bfail(b, CC_ERR_ARG, "tile variant out of range for this precision");
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    b->eng.tile_x = tile_x;
    b->eng.tile_y = tile_y;
    BHIPCHK(b, engine_plan(b->eng, b->stream));
    return CC_OK;
}

int32_t cc_batch_size(const cc_batch* b) { return b ? (int32_t)b->eng.mem.size() : 0; }

cc_status cc_batch_set_launch_mode(cc_batch* b, int32_t mode) {
    if (!b) return CC_ERR_ARG;
    if (mode != CC_LAUNCH_PER_PHASE && mode != CC_LAUNCH_PERSISTENT) return bfail(b, CC_ERR_ARG, "unknown launch mode");
    if (mode == CC_LAUNCH_PERSISTENT)
        for (cc_ctx* c : b->eng.mem)
            if (c->budget_on) return bfail(b, CC_ERR_UNSUPPORTED, "a member tracks its budget (not in the persistent mode)");
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    b->eng.mode = mode;
    BHIPCHK(b, engine_plan(b->eng, b->stream));
    return CC_OK;
}

cc_status cc_batch_step(cc_batch* b, const double* h_dt, int32_t* h_status) {
    if (!b || !h_dt) return CC_ERR_ARG;
    Engine& E = b->eng;
    int n = (int)E.mem.size();
    if (n == 0) return CC_OK;
    int buf = E.buf;
    BHIPCHK(b, engine_hostbuf(E, buf));
    for (int k = 0; k < n; k++) {
        cc_ctx* c = E.mem[k];
        cc_status st = prepare_step(c, h_dt[k], E.h_args[buf][k]);
        if (st != CC_OK) {
            b->err = "member " + std::to_string(k) + ": " + c->err;
            return st;
        }
        // the members' results land in the batch's gather arrays
        E.h_args[buf][k].cfl_out = E.d_cflout + 2 * k;
    }
    hipError_t e = hipSuccess;
    if (E.timing & 1) {
        if (E.prec == CC_FP32_GEOM64) step_sequence_timed<float>(E, b->stream, buf, -1);
        else step_sequence_timed<double>(E, b->stream, buf, -1);
        e = hipGetLastError();
    } else {
        e = E.prec == CC_FP32_GEOM64 ? engine_graph_step<float>(E, b->stream, buf, -1)
                                     : engine_graph_step<double>(E, b->stream, buf, -1);
    }
    if (e != hipSuccess) return bfail(b, CC_ERR_DEVICE, std::string("batch step: ") + hipGetErrorString(e));
    BHIPCHK(b, hipEventRecord(E.ev[buf], b->stream));
    E.ev_used[buf] = true;
    E.buf = 1 - buf;
    BHIPCHK(b, wait_event(E.ev[buf]));
    for (int k = 0; k < n; k++) {
        cc_ctx* c = E.mem[k];
        c->in_step = true;
        c->sweeps_done = 2;
        c->speeds_ready = false;
        cc_end_step(c);
        if (h_status) h_status[k] = (int32_t)E.h_gather[2 * k];
    }
    return CC_OK;
}

cc_status cc_batch_advance(cc_batch* b, int32_t nsteps, double cfl, double* h_dt, float* h_step_ms,
                           int32_t* h_done) {
    if (!b || nsteps < 0 || !(cfl > 0.0) || !std::isfinite(cfl)) return CC_ERR_ARG;
    Engine& E = b->eng;
    int n = (int)E.mem.size();
    if (h_done)
        for (int k = 0; k < n; k++) h_done[k] = 0;
    if (n == 0 || nsteps == 0) return CC_OK;
    return E.prec == CC_FP32_GEOM64 ? batch_advance<float>(b, nsteps, cfl, h_dt, h_step_ms, h_done)
                                    : batch_advance<double>(b, nsteps, cfl, h_dt, h_step_ms, h_done);
}

cc_status cc_batch_cfl_dt(cc_batch* b, double cfl, double* h_dt) {
    if (!b || !h_dt || !(cfl > 0.0)) return CC_ERR_ARG;
    Engine& E = b->eng;
    for (size_t k = 0; k < E.mem.size(); k++) {
        cc_status st = cc_cfl_dt(E.mem[k], cfl, &h_dt[k], nullptr);
        if (st != CC_OK) {
            b->err = "member " + std::to_string(k) + ": " + E.mem[k]->err;
            return st;
        }
    }
    return CC_OK;
}

cc_status cc_batch_last_dt(cc_batch* b, double cfl, double* h_dt, int32_t* h_status) {
    if (!b || !h_dt || !(cfl > 0.0)) return CC_ERR_ARG;
    Engine& E = b->eng;
    for (size_t k = 0; k < E.mem.size(); k++) {
        cc_ctx* c = E.mem[k];
        double sx, sy;
        std::memcpy(&sx, &E.h_cflout[2 * k], 8);
        std::memcpy(&sy, &E.h_cflout[2 * k + 1], 8);
        unsigned int st = E.h_gather[2 * k];
        if (h_status) h_status[k] = (int32_t)st;
        cc_status r = status_error(c, st, sx, sy);
        h_dt[k] = r == CC_OK ? dt_from_speeds(c, cfl, sx, sy) : 0.0;
    }
    return CC_OK;
}

const char* cc_batch_last_error(const cc_batch* b) { return b ? b->err.c_str() : ""; }


}  // extern "C"
