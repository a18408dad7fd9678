// Host side of the cut-cell library: context, workspace carving, body posing, level
// bookkeeping and kernel launches for the split step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/cc.h"
#include "cc_device.h"
#include "geometry.h"
#include "reduce.h"
#include "sweep.h"

using namespace cc;

namespace {

constexpr size_t ALIGN = 256;
constexpr int NPART = 1024;  // blocks of the deterministic sum
constexpr int TPB = 256;
constexpr int TPB_BOX = 64;  // small box kernels: spread a few thousand cells over all CUs

size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
    size_t nc, nvx, nfx, nfy, cap, capf;
    size_t u_bytes;
    size_t off_u[2], off_vcls[3], off_fx[3], off_fy[3], off_alpha[3], off_poly[3];
    size_t off_qb, off_stamp;
    size_t off_sQ, off_sU1, off_shas, off_sbt, off_swall, off_sfb, off_swv, off_sahat, off_sU2, off_sgone;
    size_t off_sf1, off_sf2, off_nbad;
    size_t off_smax, off_status, off_ncol, off_part, off_tot;
    size_t total;
    int capw, caph;
};

int body_m(const cc_body* b) { return b && b->nverts > 0 && b->verts ? b->nverts : 0; }

Layout make_layout(const cc_config* c, const cc_body* b) {
    Layout L{};
    size_t nx = c->nx, ny = c->ny;
    int m = body_m(b);
    L.nc = nx * ny;
    L.nvx = (nx + 1) * (ny + 1);
    L.nfx = ny * (nx + 1);
    L.nfy = (ny + 1) * nx;
    size_t rs = c->precision == CC_FP32_GEOM64 ? sizeof(float) : sizeof(double);
    L.u_bytes = 4 * L.nc * rs;
    // staging capacity: the body stays inside a disc of radius R about its moving origin
    double R = 0.0;
    for (int k = 0; k < m; k++) R = std::max(R, std::hypot(b->verts[2 * k], b->verts[2 * k + 1]));
    double hx = (c->x_hi - c->x_lo) / c->nx, hy = (c->y_hi - c->y_lo) / c->ny;
    if (m > 0) {
        double cw = std::ceil(2.0 * R / hx) + 16.0, ch = std::ceil(2.0 * R / hy) + 16.0;
        L.capw = (int)std::min<double>(cw, (double)nx);
        L.caph = (int)std::min<double>(ch, (double)ny);
    } else {
        L.capw = L.caph = 0;
    }
    L.cap = (size_t)L.capw * L.caph;
    L.capf = m > 0 ? (size_t)(L.capw + 1) * (L.caph + 1) : 0;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += up(bytes);
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
    L.off_qb = take(m > 0 ? 4 * L.nc * 8 : 8);
    L.off_stamp = take(m > 0 ? L.nc * 4 : 4);
    size_t cap = std::max<size_t>(L.cap, 1), capf = std::max<size_t>(L.capf, 1);
    L.off_sQ = take(4 * cap * 8);
    L.off_sU1 = take(4 * cap * 8);
    L.off_shas = take(cap);
    L.off_sbt = take(capf * 8);
    L.off_swall = take(cap);
    L.off_sfb = take(4 * cap * 8);
    L.off_swv = take(4 * cap * 8);
    L.off_sahat = take(cap * 8);
    L.off_sU2 = take(4 * cap * 8);
    L.off_sgone = take(cap);
    L.off_sf1 = take(cap);
    L.off_sf2 = take(cap);
    L.off_nbad = take(8);
    L.off_smax = take(16);
    L.off_status = take(4);
    L.off_ncol = take(4);
    L.off_part = take(4 * NPART * 8);
    L.off_tot = take(4 * 8);
    L.total = o;
    return L;
}

struct TimedPair {
    hipEvent_t a, b;
    int kind;
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
    // state
    int cur;  // U[cur] holds the level-n (or current) state
    // levels
    Level lev[3];
    Box lbox[3];        // region of each slot that may differ from all-fluid
    double* hpoly[3];   // pinned host copies of the posed polygons
    hipEvent_t poly_ev[3];
    bool poly_ev_valid[3];
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
    // timing
    bool timing;
    std::vector<TimedPair> pending, pool;
    double tsum[4];
    double tcnt[4];
    std::string err;
};

namespace {

thread_local std::string g_create_err;  // message of the last failed cc_create on this thread

cc_status fail(cc_ctx* c, cc_status s, const std::string& msg) {
    if (c) c->err = msg;
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

template <typename T>
T* at(cc_ctx* c, size_t off) {
    return reinterpret_cast<T*>(c->ws + off);
}

bool fp32(const cc_ctx* c) { return c->cfg.precision == CC_FP32_GEOM64; }

void pose(const cc_ctx* c, double t, double* out) {
    double th = c->theta0 + c->amp * std::sin(c->omega * t);
    double cs = std::cos(th), sn = std::sin(th);
    double cx = c->ref_x + c->vx * t, cy = c->ref_y + c->vy * t;
    for (int k = 0; k < c->m; k++) {
        double bx = c->bverts[2 * k], by = c->bverts[2 * k + 1];
        out[2 * k] = (cs * bx - sn * by) + cx;
        out[2 * k + 1] = (sn * bx + cs * by) + cy;
    }
}

// Bounding box, certificate discs and cell box of a posed polygon.
void poly_info(const cc_ctx* c, const double* pv, Poly& P, Box& cells) {
    int m = c->m;
    P.m = m;
    P.xmin = P.ymin = INFINITY;
    P.xmax = P.ymax = -INFINITY;
    for (int k = 0; k < m; k++) {
        P.xmin = std::fmin(P.xmin, pv[2 * k]);
        P.xmax = std::fmax(P.xmax, pv[2 * k]);
        P.ymin = std::fmin(P.ymin, pv[2 * k + 1]);
        P.ymax = std::fmax(P.ymax, pv[2 * k + 1]);
    }
    P.rin2 = -1.0;
    P.rout2 = 0.0;
    P.cx = P.cy = 0.0;
    if (m >= 8) {
        double sx = 0.0, sy = 0.0;
        for (int k = 0; k < m; k++) {
            sx += pv[2 * k];
            sy += pv[2 * k + 1];
        }
        double cx = sx / m, cy = sy / m;
        double rin = INFINITY, rout = 0.0;
        for (int k = 0; k < m; k++) {
            int k1 = (k + 1) % m;
            double ex = pv[2 * k1] - pv[2 * k], ey = pv[2 * k1 + 1] - pv[2 * k + 1];
            double len = std::hypot(ex, ey);
            if (len > 0.0) {
                double sd = (ex * (cy - pv[2 * k + 1]) - ey * (cx - pv[2 * k])) / len;
                rin = std::min(rin, sd);
            }
            rout = std::max(rout, std::hypot(pv[2 * k] - cx, pv[2 * k + 1] - cy));
        }
        if (rin > 1e-7 * rout && std::isfinite(rin)) {
            P.cx = cx;
            P.cy = cy;
            P.rin2 = (rin * (1.0 - 1e-6)) * (rin * (1.0 - 1e-6));
            P.rout2 = (rout * (1.0 + 1e-6)) * (rout * (1.0 + 1e-6));
        }
    }
    if (m == 0 || P.xmax < c->cfg.x_lo || P.xmin > c->cfg.x_hi || P.ymax < c->cfg.y_lo || P.ymin > c->cfg.y_hi) {
        cells = Box{0, 0, 0, 0};
        return;
    }
    int i0 = (int)std::floor((P.xmin - c->cfg.x_lo) / c->hx) - 2;
    int i1 = (int)std::floor((P.xmax - c->cfg.x_lo) / c->hx) + 3;
    int j0 = (int)std::floor((P.ymin - c->cfg.y_lo) / c->hy) - 2;
    int j1 = (int)std::floor((P.ymax - c->cfg.y_lo) / c->hy) + 3;
    cells.i0 = std::max(i0, 0);
    cells.i1 = std::min(i1, c->g.nx);
    cells.j0 = std::max(j0, 0);
    cells.j1 = std::min(j1, c->g.ny);
    if (cells.i0 >= cells.i1 || cells.j0 >= cells.j1) cells = Box{0, 0, 0, 0};
}

bool box_empty(const Box& b) { return b.i0 >= b.i1 || b.j0 >= b.j1; }

Box box_union(const Box& a, const Box& b) {
    if (box_empty(a)) return b;
    if (box_empty(b)) return a;
    return Box{std::min(a.i0, b.i0), std::max(a.i1, b.i1), std::min(a.j0, b.j0), std::max(a.j1, b.j1)};
}

unsigned nblk(size_t n, int t = TPB) { return (unsigned)((n + t - 1) / t); }


void tstart(cc_ctx* c, int kind, TimedPair& tp) {
    if (!c->timing) return;
    if (c->pool.empty()) {
        TimedPair p;
        (void)hipEventCreate(&p.a);
        (void)hipEventCreate(&p.b);
        c->pool.push_back(p);
    }
    tp = c->pool.back();
    c->pool.pop_back();
    tp.kind = kind;
    (void)hipEventRecord(tp.a, c->stream);
}
void tstop(cc_ctx* c, TimedPair& tp) {
    if (!c->timing) return;
    (void)hipEventRecord(tp.b, c->stream);
    c->pending.push_back(tp);
}

// Compute the geometry of a posed polygon into a slot (device), over the union of the
// slot's previous region and the polygon's box.
cc_status compute_level(cc_ctx* c, int slot, const double* pv) {
    Level& L = c->lev[slot];
    Box cells;
    poly_info(c, pv, L.poly, cells);
    if (c->m > 0) {
        if (c->poly_ev_valid[slot]) HIPCHK(c, hipEventSynchronize(c->poly_ev[slot]));
        std::memcpy(c->hpoly[slot], pv, sizeof(double) * 2 * c->m);
        HIPCHK(c, hipMemcpyAsync((void*)L.poly.v, c->hpoly[slot], sizeof(double) * 2 * c->m, hipMemcpyHostToDevice,
                                 c->stream));
        HIPCHK(c, hipEventRecord(c->poly_ev[slot], c->stream));
        c->poly_ev_valid[slot] = true;
    }
    Box reg = box_union(c->lbox[slot], cells);
    c->lbox[slot] = cells;
    if (box_empty(reg)) return CC_OK;
    TimedPair tp{};
    tstart(c, 3, tp);
    int vw = reg.w() + 1, vh = reg.h() + 1;
    hipLaunchKernelGGL(k_geo_vertices, dim3(nblk((size_t)vw * vh, ITEMS_PER_BLOCK)), dim3(TPB), 0, c->stream, c->g, L,
                       reg.i0, reg.j0, vw, vh);
    size_t nf = (size_t)vw * (vh - 1) + (size_t)(vw - 1) * vh;
    hipLaunchKernelGGL(k_geo_faces, dim3(nblk(nf, ITEMS_PER_BLOCK)), dim3(TPB), 0, c->stream, c->g, L, reg.i0, reg.j0,
                       vw, vh);
    hipLaunchKernelGGL(k_geo_cells, dim3(nblk((size_t)reg.w() * reg.h(), ITEMS_PER_BLOCK)), dim3(TPB), 0, c->stream,
                       c->g, L, reg.i0, reg.j0, reg.w(), reg.h());
    tstop(c, tp);
    HIPCHK(c, hipGetLastError());
    return CC_OK;
}

template <typename R>
cc_status run_sweep(cc_ctx* c, int dir, double dt, bool first) {
    const Level& Ls = c->lev[first ? c->s0 : c->sm];
    const Level& Le = c->lev[first ? c->sm : c->s1];
    Box ub = box_union(c->lbox[first ? c->s0 : c->sm], c->lbox[first ? c->sm : c->s1]);
    Box B{0, 0, 0, 0};
    if (!box_empty(ub)) {
        B.i0 = std::max(ub.i0 - 3, 0);
        B.i1 = std::min(ub.i1 + 3, c->g.nx);
        B.j0 = std::max(ub.j0 - 3, 0);
        B.j1 = std::min(ub.j1 + 3, c->g.ny);
        if ((size_t)B.w() > (size_t)c->lay.capw || (size_t)B.h() > (size_t)c->lay.caph)
            return fail(c, CC_ERR_WORKSPACE, "sweep region exceeds the staging capacity");
    }
    c->last_sweep_box = B;
    size_t nc = c->lay.nc;
    const R* Uin = at<R>(c, c->lay.off_u[c->cur]);
    R* Uout = at<R>(c, c->lay.off_u[1 - c->cur]);
    double h = dir == 0 ? c->hx : c->hy;
    double lam = dt / h;
    Stage S;
    S.Q = at<double>(c, c->lay.off_sQ);
    S.U1 = at<double>(c, c->lay.off_sU1);
    S.has = at<int8_t>(c, c->lay.off_shas);
    S.bt = at<double>(c, c->lay.off_sbt);
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
    Common C{at<double>(c, c->lay.off_qb), at<int32_t>(c, c->lay.off_stamp)};
    unsigned int* status = at<unsigned int>(c, c->lay.off_status);
    unsigned int* ncol = at<unsigned int>(c, c->lay.off_ncol);
    size_t nb = (size_t)B.w() * B.h();
    int32_t step_id = (int32_t)(c->step & 0x7fffffff);
    TimedPair tb{};
    if (nb > 0) {
        tstart(c, 2, tb);
        size_t nf = dir == 0 ? (size_t)(B.w() + 1) * B.h() : (size_t)B.w() * (B.h() + 1);
        if (dir == 0)
            hipLaunchKernelGGL(k_swept<0>, dim3(nblk(nf, ITEMS_PER_BLOCK)), dim3(TPB), 0, c->stream, c->g, Ls, Le,
                               c->mot, B, S);
        else
            hipLaunchKernelGGL(k_swept<1>, dim3(nblk(nf, ITEMS_PER_BLOCK)), dim3(TPB), 0, c->stream, c->g, Ls, Le,
                               c->mot, B, S);
        hipLaunchKernelGGL(k_stage<R>, dim3(nblk(nb, TPB_BOX)), dim3(TPB_BOX), 0, c->stream, c->g, Ls, Le, Uin, B, S, status);
        if (dir == 0)
            hipLaunchKernelGGL(k_wall<0>, dim3(nblk(nb, TPB_BOX)), dim3(TPB_BOX), 0, c->stream, c->g, Ls, Le, c->mot, B, S, C,
                               (int)first, step_id);
        else
            hipLaunchKernelGGL(k_wall<1>, dim3(nblk(nb, TPB_BOX)), dim3(TPB_BOX), 0, c->stream, c->g, Ls, Le, c->mot, B, S, C,
                               (int)first, step_id);
        tstop(c, tb);
    }
    TimedPair td{};
    tstart(c, dir, td);
    if (dir == 0) {
        dim3 grid((unsigned)((c->g.nx + DX_OUT - 1) / DX_OUT), (unsigned)c->g.ny);
        hipLaunchKernelGGL((k_dense_x<R, R>), grid, dim3(DX_T), 0, c->stream, c->g, Uin, Uout, B, (R)lam);
    } else {
        // rows per thread: enough column segments to give every CU several wavefronts
        long long cells = (long long)c->g.nx * c->g.ny;
        int rows = (int)std::max<long long>(4, std::min<long long>(64, cells / (256LL * 256 * 4)));
        dim3 grid((unsigned)((c->g.nx + 255) / 256), (unsigned)((c->g.ny + rows - 1) / rows));
        hipLaunchKernelGGL((k_dense_y<R, R>), grid, dim3(256), 0, c->stream, c->g, Uin, Uout, B, (R)lam, rows);
    }
    tstop(c, td);
    if (nb > 0) {
        tstart(c, 2, tb);
        if (dir == 0)
            hipLaunchKernelGGL((k_patch<0, R>), dim3(nblk(nb, TPB_BOX)), dim3(TPB_BOX), 0, c->stream, c->g, Ls, Le, Uin, B, S, lam,
                               ncol);
        else
            hipLaunchKernelGGL((k_patch<1, R>), dim3(nblk(nb, TPB_BOX)), dim3(TPB_BOX), 0, c->stream, c->g, Ls, Le, Uin, B, S, lam,
                               ncol);
        hipLaunchKernelGGL(k_cover<R>, dim3(nblk(nb, TPB_BOX)), dim3(TPB_BOX), 0, c->stream, c->g, Le, B, S, Uout);
        // collapse rounds after covering: the content ping-pongs U1 -> Q -> Uout
        hipLaunchKernelGGL(k_fix<R>, dim3(nblk(nb, TPB_BOX)), dim3(TPB_BOX), 0, c->stream, c->g, Le, B, S, 0,
                           (const double*)S.U1, (const int8_t*)S.f1, S.Q, S.f2, Uout, ncol, status);
        hipLaunchKernelGGL(k_fix<R>, dim3(nblk(nb, TPB_BOX)), dim3(TPB_BOX), 0, c->stream, c->g, Le, B, S, 1,
                           (const double*)S.Q, (const int8_t*)S.f2, (double*)nullptr, (int8_t*)nullptr, Uout, ncol,
                           status);
        tstop(c, tb);
    }
    (void)nc;
    HIPCHK(c, hipGetLastError());
    c->cur = 1 - c->cur;
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

}  // namespace

extern "C" {

size_t cc_workspace_bytes(const cc_config* cfg, const cc_body* body) {
    if (!cfg || cfg->nx < 1 || cfg->ny < 1) return 0;
    return make_layout(cfg, body).total;
}

cc_status cc_create(const cc_config* cfg, const cc_body* body, void* d_ws, size_t ws_bytes, void* hip_stream,
                    cc_ctx** out) {
    if (!out) return create_fail(nullptr, CC_ERR_ARG, "null output pointer");
    *out = nullptr;
    if (!cfg || cfg->nx < 1 || cfg->ny < 1 || !(cfg->x_hi > cfg->x_lo) || !(cfg->y_hi > cfg->y_lo) ||
        !(cfg->gamma > 1.0) || cfg->reserved != 0 || (cfg->precision != CC_FP64 && cfg->precision != CC_FP32_GEOM64) ||
        !(cfg->alpha_min >= 0.0 && cfg->alpha_min < 0.5))
        return create_fail(nullptr, CC_ERR_ARG, "invalid configuration");
    for (int k = 0; k < 4; k++)
        if (cfg->bc[k] != CC_BC_TRANSMISSIVE && cfg->bc[k] != CC_BC_REFLECTIVE)
            return create_fail(nullptr, CC_ERR_ARG, "invalid boundary condition");
    if (body && body->nverts > 0 && !body->verts) return create_fail(nullptr, CC_ERR_ARG, "body without vertices");
    Layout lay = make_layout(cfg, body);
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
    c->m = body_m(body);
    if (c->m > 0) {
        c->bverts.assign(body->verts, body->verts + 2 * c->m);
        c->ref_x = body->ref_x;
        c->ref_y = body->ref_y;
        c->theta0 = body->theta0;
        c->vx = body->vx;
        c->vy = body->vy;
        c->amp = body->pitch_amp;
        c->omega = body->pitch_omega;
    }
    c->cur = 0;
    c->s0 = 0;
    c->sm = 1;
    c->s1 = 2;
    for (int s = 0; s < 3; s++) {
        Level& L = c->lev[s];
        L.vcls = at<int8_t>(c, lay.off_vcls[s]);
        L.fx = at<double2>(c, lay.off_fx[s]);
        L.fy = at<double2>(c, lay.off_fy[s]);
        L.alpha = at<double>(c, lay.off_alpha[s]);
        L.poly = Poly{at<double>(c, lay.off_poly[s]), 0, 0, 0, 0, 0, 0, 0, -1.0, 0.0};
        c->lbox[s] = Box{0, 0, 0, 0};
        c->hpoly[s] = nullptr;
        c->poly_ev_valid[s] = false;
        if (c->m > 0) {
            hipError_t e1 = hipHostMalloc((void**)&c->hpoly[s], sizeof(double) * 2 * c->m, hipHostMallocDefault);
            if (e1 != hipSuccess) return create_fail(c, CC_ERR_DEVICE, std::string("hipHostMalloc: ") + hipGetErrorString(e1));
            hipError_t e2 = hipEventCreateWithFlags(&c->poly_ev[s], hipEventDisableTiming);
            if (e2 != hipSuccess) {
                (void)hipHostFree(c->hpoly[s]);
                c->hpoly[s] = nullptr;
                return create_fail(c, CC_ERR_DEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e2));
            }
        }
    }
    // all-fluid levels, clean reductions, stamps that match no step
    hipError_t e = hipSuccess;
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
    if (e == hipSuccess && c->m > 0) e = hipMemsetAsync(at<int32_t>(c, lay.off_stamp), 0xff, lay.nc * 4, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + lay.off_smax, 0, 16, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + lay.off_status, 0, 4, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->ws + lay.off_ncol, 0, 4, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return create_fail(c, CC_ERR_DEVICE, std::string("initialisation: ") + hipGetErrorString(e));
    *out = c;
    return CC_OK;
}


cc_status cc_destroy(cc_ctx* c) {
    if (!c) return CC_ERR_ARG;
    (void)hipStreamSynchronize(c->stream);
    for (int s = 0; s < 3; s++) {
        if (c->hpoly[s]) {
            (void)hipHostFree(c->hpoly[s]);
            (void)hipEventDestroy(c->poly_ev[s]);
        }
    }
    for (auto& p : c->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto& p : c->pool) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    delete c;
    return CC_OK;
}

const char* cc_last_error(const cc_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

cc_status cc_geometry(cc_ctx* c, double t, int32_t level) {
    if (!c || level < 0 || level > 2) return fail(c, CC_ERR_ARG, "bad level");
    if (c->in_step) return fail(c, CC_ERR_ARG, "cc_geometry inside a step");
    int slot = level == 0 ? c->s0 : level == 1 ? c->sm : c->s1;
    std::vector<double> pv(2 * std::max(c->m, 1));
    pose(c, t, pv.data());
    return compute_level(c, slot, pv.data());
}

cc_status cc_geometry_dump(cc_ctx* c, int32_t level, int8_t* d_vcls, double* d_alpha, double* d_bx, double* d_by) {
    if (!c || level < 0 || level > 2) return fail(c, CC_ERR_ARG, "bad level");
    int slot = level == 0 ? c->s0 : level == 1 ? c->sm : c->s1;
    const Level& L = c->lev[slot];
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
    c->in_step = false;
    c->t = t0;
    c->step = 0;
    c->parity = 0;
    c->cur = 0;
    cc_status st = cc_geometry(c, t0, 0);
    if (st != CC_OK) return st;
    const double* al = c->lev[c->s0].alpha;
    if (fp32(c))
        hipLaunchKernelGGL(k_prim_to_u<float>, dim3(nblk(c->lay.nc)), dim3(TPB), 0, c->stream, c->g, al, d_prim,
                           at<float>(c, c->lay.off_u[0]));
    else
        hipLaunchKernelGGL(k_prim_to_u<double>, dim3(nblk(c->lay.nc)), dim3(TPB), 0, c->stream, c->g, al, d_prim,
                           at<double>(c, c->lay.off_u[0]));
    HIPCHK(c, hipMemsetAsync(c->ws + c->lay.off_status, 0, 4, c->stream));
    HIPCHK(c, hipMemsetAsync(c->ws + c->lay.off_ncol, 0, 4, c->stream));
    if (c->m > 0) HIPCHK(c, hipMemsetAsync(c->ws + c->lay.off_stamp, 0xff, c->lay.nc * 4, c->stream));
    HIPCHK(c, hipGetLastError());
    c->have_state = true;
    return CC_OK;
}

cc_status cc_set_clock(cc_ctx* c, double t, int64_t step) {
    if (!c || step < 0 || !std::isfinite(t)) return fail(c, CC_ERR_ARG, "bad argument");
    c->in_step = false;
    c->t = t;
    c->step = step;
    c->parity = (int)(step & 1);
    cc_status st = cc_geometry(c, t, 0);
    if (st != CC_OK) return st;
    if (c->m > 0) HIPCHK(c, hipMemsetAsync(c->ws + c->lay.off_stamp, 0xff, c->lay.nc * 4, c->stream));
    return CC_OK;
}

cc_status cc_set_u(cc_ctx* c, const double* d_u) {
    if (!c || !d_u) return fail(c, CC_ERR_ARG, "null argument");
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
    if (!c->have_state) return fail(c, CC_ERR_ARG, "no state set");
    if (c->in_step) return fail(c, CC_ERR_ARG, "step already begun");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, CC_ERR_MOTION, "dt must be positive");
    double t1 = c->t + dt;
    int m = std::max(c->m, 1);
    std::vector<double> p0(2 * m), p1(2 * m), pm(2 * m);
    pose(c, c->t, p0.data());
    pose(c, t1, p1.data());
    for (int k = 0; k < c->m; k++) {
        if (c->parity == 0) {
            pm[2 * k] = p1[2 * k];
            pm[2 * k + 1] = p0[2 * k + 1];
        } else {
            pm[2 * k] = p0[2 * k];
            pm[2 * k + 1] = p1[2 * k + 1];
        }
    }
    cc_status st = check_motion(c, p0, p1);
    if (st != CC_OK) return st;
    st = compute_level(c, c->sm, pm.data());
    if (st != CC_OK) return st;
    st = compute_level(c, c->s1, p1.data());
    if (st != CC_OK) return st;
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
    c->in_step = true;
    c->sweeps_done = 0;
    c->step_dt = dt;
    return CC_OK;
}

cc_status cc_sweep(cc_ctx* c, int32_t dir, double dt) {
    if (!c) return CC_ERR_ARG;
    if (!c->in_step || c->sweeps_done > 1) return fail(c, CC_ERR_ARG, "cc_sweep outside a step");
    int want = c->sweeps_done == 0 ? c->parity : 1 - c->parity;
    if (dir != want) return fail(c, CC_ERR_ARG, "sweep direction out of order");
    if (dt != c->step_dt) return fail(c, CC_ERR_ARG, "dt differs from cc_begin_step");
    bool first = c->sweeps_done == 0;
    cc_status st = fp32(c) ? run_sweep<float>(c, dir, dt, first) : run_sweep<double>(c, dir, dt, first);
    if (st != CC_OK) return st;
    c->sweeps_done++;
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

cc_status cc_step(cc_ctx* c, double dt) {
    cc_status st = cc_begin_step(c, dt);
    if (st != CC_OK) return st;
    int d1 = c->parity, d2 = 1 - c->parity;
    if ((st = cc_sweep(c, d1, dt)) != CC_OK) return st;
    if ((st = cc_sweep(c, d2, dt)) != CC_OK) return st;
    return cc_end_step(c);
}

cc_status cc_cfl_dt(cc_ctx* c, double cfl, double* h_dt) {
    if (!c || !h_dt || !(cfl > 0.0)) return fail(c, CC_ERR_ARG, "bad argument");
    if (c->in_step) return fail(c, CC_ERR_ARG, "cc_cfl_dt inside a step");
    unsigned long long* smax = at<unsigned long long>(c, c->lay.off_smax);
    unsigned long long* part = at<unsigned long long>(c, c->lay.off_part);
    const double* al = c->lev[c->s0].alpha;
    if (fp32(c))
        hipLaunchKernelGGL(k_cfl<float>, dim3(CFL_BLOCKS), dim3(256), 0, c->stream, c->g, al,
                           at<float>(c, c->lay.off_u[c->cur]), part);
    else
        hipLaunchKernelGGL(k_cfl<double>, dim3(CFL_BLOCKS), dim3(256), 0, c->stream, c->g, al,
                           at<double>(c, c->lay.off_u[c->cur]), part);
    hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(256), 0, c->stream, CFL_BLOCKS, (const unsigned long long*)part, smax);
    HIPCHK(c, hipGetLastError());
    unsigned long long hs[2];
    unsigned int status = 0;
    HIPCHK(c, hipMemcpyAsync(hs, smax, 16, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&status, c->ws + c->lay.off_status, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double sx, sy;
    std::memcpy(&sx, &hs[0], 8);
    std::memcpy(&sy, &hs[1], 8);
    if (status & 1u) return fail(c, CC_ERR_STATE, "a cell became fluid without donor neighbours");
    if (status & 2u) return fail(c, CC_ERR_STATE, "a cut cell stayed inadmissible after two collapse rounds");
    if (!std::isfinite(sx) || !std::isfinite(sy)) return fail(c, CC_ERR_STATE, "non-finite or non-physical state");
    if (c->m > 0) {
        std::vector<double> pv(2 * c->m);
        pose(c, c->t, pv.data());
        double thd = c->amp * c->omega * std::cos(c->omega * c->t);
        double cx = c->ref_x + c->vx * c->t, cy = c->ref_y + c->vy * c->t;
        for (int k = 0; k < c->m; k++) {
            double ux = c->vx - thd * (pv[2 * k + 1] - cy);
            double uy = c->vy + thd * (pv[2 * k] - cx);
            sx = std::fmax(sx, std::fabs(ux));
            sy = std::fmax(sy, std::fabs(uy));
        }
    }
    *h_dt = cfl * std::fmin(c->hx / sx, c->hy / sy);
    return CC_OK;
}

cc_status cc_totals(cc_ctx* c, double* h_totals4) {
    if (!c || !h_totals4) return fail(c, CC_ERR_ARG, "bad argument");
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
    hipLaunchKernelGGL(k_sum_final, dim3(4), dim3(RT), 0, c->stream, NPART, (const double*)part, tot);
    HIPCHK(c, hipGetLastError());
    double h[4];
    HIPCHK(c, hipMemcpyAsync(h, tot, 32, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double area = c->hx * c->hy;
    for (int k = 0; k < 4; k++) h_totals4[k] = h[k] * area;
    return CC_OK;
}

cc_status cc_info(cc_ctx* c, double* h_out, int32_t n) {
    if (!c || !h_out || n < 1) return fail(c, CC_ERR_ARG, "bad argument");
    unsigned int dev[2];
    HIPCHK(c, hipMemcpyAsync(&dev[0], c->ws + c->lay.off_status, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&dev[1], c->ws + c->lay.off_ncol, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double v[8] = {c->t, (double)c->step, (double)c->parity, (double)dev[0], (double)dev[1],
                   (double)c->last_sweep_box.w() * c->last_sweep_box.h(), (double)c->lay.cap, 0.0};
    for (int k = 0; k < n && k < 8; k++) h_out[k] = v[k];
    return CC_OK;
}

cc_status cc_timing(cc_ctx* c, int32_t enable) {
    if (!c) return CC_ERR_ARG;
    c->timing = enable != 0;
    return CC_OK;
}

cc_status cc_timing_read(cc_ctx* c, double* h_out, int32_t n) {
    if (!c || !h_out) return fail(c, CC_ERR_ARG, "bad argument");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double sum[4] = {0, 0, 0, 0}, cnt[4] = {0, 0, 0, 0};
    for (auto& p : c->pending) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, p.a, p.b));
        sum[p.kind] += ms;
        cnt[p.kind] += 1.0;
        c->pool.push_back(p);
    }
    c->pending.clear();
    for (int k = 0; k < 4 && 2 * k + 1 < n; k++) {
        h_out[2 * k] = sum[k];
        h_out[2 * k + 1] = cnt[k];
    }
    return CC_OK;
}

}  // extern "C"
