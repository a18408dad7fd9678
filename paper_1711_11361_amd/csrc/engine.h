// Launch wrappers: every phase of a split step is one kernel launch over all instances of
// a batch (one instance for a single context).  The per-step arguments of each instance
// live in device memory (StepArgs, uploaded once per step), so the launches themselves
// have fixed grids and fixed arguments and can be captured in a HIP graph.  Blocks are
// mapped to (instance, block within the instance) through per-launch offset tables sized
// from each instance's capacities; blocks beyond the work of the current step exit.
#pragma once
#include "cc_device.h"
#include "geometry.h"
#include "reduce.h"
#include "sweep.h"
#include "bodies.h"

namespace cc {

struct PlanConst;
struct PlanState;

struct StepArgs {
    Grid g;
    GeoJob geo[2];   // stage level and end level of the step
    SweepJob sw[2];  // first and second sweep
    Motion mot;
    const Motion* bmot;  // several bodies: each body's motion (null for one body)
    double dt;           // the step's time step (host-planned steps; the axisymmetric source)
    Stage S;
    Common C;
    unsigned int* status;
    unsigned int* ncol;
    double* bt[2];  // time-averaged apertures of each sweep (box-local faces)
    int nb_cells, nb_swept;  // blocks of the cell stage (both levels) and of one sweep's apertures
    int32_t step_id;
    // wave-speed maxima of the state after the step
    unsigned long long* cfl_out;   // 2: max (|u|+a) along x and y, as bit patterns
    unsigned long long* spd;       // partial maxima of a captured step: NSPD slot pairs the dense
    int spd_dense;                 // tiles of the second sweep share, then (from pair spd_dense
                                   // on) a pair per box block
    // a device-planned run: the block that combines the wave speeds also plans the next
    // step (null otherwise)
    const PlanConst* pc;
    PlanState* ps;
    double* dtlog;
    // conservation budget (bs.base null: not tracked): per-sweep slots, and the running
    // sums since the state was set: domain-boundary fluxes, wall terms, residuals without
    // recipients (4 components each, times the cell area)
    BudgetSlots bs;
    double* budget;
};

__device__ __forceinline__ void plan_block(const PlanConst* PC, PlanState* PS, StepArgs* out, double* dt_log);

// Launch kinds and their block sizes.
enum LaunchKind {
    L_POSE, L_V1, L_F1, L_C1,  // geometry stages (both level jobs)
    L_S1, L_BOX, L_DX, L_DY,  // sweeps
    L_CS,  // volume fractions of both levels and the apertures of both sweeps
    L_BOXW,  // box cells, T_WIDE per block (launched beside the dense tiles)
    L_PX, L_PY,  // the patch update's blocks: box line segments (x sweep), column tiles (y sweep)
    NKINDS
};
constexpr int T_WIDE = 256;  // geometry and aperture stages, dense, time step
constexpr int T_BOX = 64;    // box phases: a few thousand cells spread over all CUs

__device__ __forceinline__ int find_unit(const int* __restrict__ off, int n, int b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct Unit {
    int u, lb, nb;  // unit, block within the unit, blocks of the unit
};
// Unit of block b of a launch.
__device__ __forceinline__ Unit unit_at(const int* __restrict__ off, int n, int b) {
    Unit r;
    r.u = n == 1 ? 0 : find_unit(off, n, b);
    r.lb = b - off[r.u];
    r.nb = off[r.u + 1] - off[r.u];
    return r;
}
__device__ __forceinline__ Unit unit_of(const int* __restrict__ off, int n) { return unit_at(off, n, blockIdx.x); }

// ------------------------------------------------------------------ geometry
// Level job lev: pose the polygon (thread t of its vertices).
__device__ __forceinline__ void pose_body(const StepArgs& a, int lev, int t) {
    const GeoJob& J = a.geo[lev];
    if (!J.active) return;
    geo_pose(J, t);
}

// Stage arrays of sweep s (the apertures are per sweep, the rest is shared).
__device__ __forceinline__ Stage stage_of(const StepArgs& a, int s) {
    Stage S = a.S;
    S.bt = a.bt[s];
    return S;
}

// The polygon of a block, staged in LDS (at most LDS_VERTS vertices, which cc_create
// checks; every item of the block left to an edge loop or a chain search reads it many
// times).  A thread has four vertex loads (16 bytes each) in flight at a time.
constexpr int LDS_VERTS = 2048;
constexpr size_t POLY_LDS = (size_t)2 * LDS_VERTS * sizeof(double);
__device__ __forceinline__ Poly stage_poly(const Poly& P, double* spoly) {
    Poly Q = P;
    const double2* src = reinterpret_cast<const double2*>(P.v);
    double2* dst = reinterpret_cast<double2*>(spoly);
    int m = P.m, nt = blockDim.x;
    for (int k0 = threadIdx.x; k0 < m; k0 += 4 * nt) {
        int k1 = k0 + nt, k2 = k0 + 2 * nt, k3 = k0 + 3 * nt;
        double2 a0 = src[k0], a1, a2, a3;
        if (k1 < m) a1 = src[k1];
        if (k2 < m) a2 = src[k2];
        if (k3 < m) a3 = src[k3];
        dst[k0] = a0;
        if (k1 < m) dst[k1] = a1;
        if (k2 < m) dst[k2] = a2;
        if (k3 < m) dst[k3] = a3;
    }
    __syncthreads();
    Q.v = spoly;
    return Q;
}

// The polygon of level job J posed in LDS, with the same formula as the copy in the level.
__device__ __forceinline__ Poly pose_lds(const GeoJob& J, double* spoly) {
    Poly Q = J.L.poly;
    const double2* src = reinterpret_cast<const double2*>(J.body);
    double2* dst = reinterpret_cast<double2*>(spoly);
    int m = Q.m, nt = blockDim.x;
    auto pose = [&](double2 b) {
        return make_double2((J.cs_x * b.x - J.sn_x * b.y) + J.cx_x, (J.sn_y * b.x + J.cs_y * b.y) + J.cy_y);
    };
    for (int k0 = threadIdx.x; k0 < m; k0 += 4 * nt) {
        int k1 = k0 + nt, k2 = k0 + 2 * nt, k3 = k0 + 3 * nt;
        double2 a0 = src[k0], a1, a2, a3;
        if (k1 < m) a1 = src[k1];
        if (k2 < m) a2 = src[k2];
        if (k3 < m) a3 = src[k3];
        dst[k0] = pose(a0);
        if (k1 < m) dst[k1] = pose(a1);
        if (k2 < m) dst[k2] = pose(a2);
        if (k3 < m) dst[k3] = pose(a3);
    }
    __syncthreads();
    Q.v = spoly;
    return Q;
}

// Items of one block left to a polygon walk, walked one at a time by a whole wavefront (all
// 64 lanes sharing the polygon's edges).  The block's items are listed in LDS (wavefront by
// wavefront, lanes in order) and dealt round-robin to its wavefronts, so a wavefront whose
// lanes drew several boundary items shares them with the others: the slowest wavefront
// walks ceil(items / wavefronts) of them.  Every thread of the block (at most T_WIDE)
// calls it.  walk(item, lane).
// The block's items with need set, listed in LDS (wavefront by wavefront, lanes in order);
// returns their count.  Every thread of the block calls it.
__device__ __forceinline__ int list_left(bool need, int t, int* items) {
    __shared__ int wcount[T_WIDE / WAVE];
    int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    unsigned long long mask = __ballot(need);
    if (lane == 0) wcount[wv] = __popcll(mask);
    __syncthreads();
    int base = 0, total = 0;
    for (int k = 0; k < nw; k++) {
        int c = wcount[k];
        base += k < wv ? c : 0;
        total += c;
    }
    if (need) items[base + __popcll(mask & ((1ull << lane) - 1ull))] = t;
    __syncthreads();
    return total;
}
template <class W>
__device__ __forceinline__ void walk_left(bool need, int t, W&& walk) {
    __shared__ int items[T_WIDE];
    int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    int total = list_left(need, t, items);
    for (int q = wv; q < total; q += nw) walk(items[q], lane);
    __syncthreads();  // the list may be rebuilt by the next call
}
// The same list taken one item per thread, packed into the block's first wavefronts (so that
// few lanes of a wavefront idle beside the ones with items).  each(item).
template <class E>
__device__ __forceinline__ void each_left(bool need, int t, E&& each) {
    __shared__ int items[T_WIDE];
    int total = list_left(need, t, items);
    if ((int)threadIdx.x < total) each(items[threadIdx.x]);
    __syncthreads();  // the list may be rebuilt by the next call
}

// Item of lane l of wavefront w among the W wavefronts of a job's nb blocks: lanes take
// items W apart, so items next to each other (the items left to walks cluster along the
// boundary) fall to different wavefronts.
__device__ __forceinline__ int spread_item(int lb, int nb) {
    int waves = nb * (T_WIDE / WAVE);
    return (int)(threadIdx.x & (WAVE - 1)) * waves + lb * (T_WIDE / WAVE) + (int)(threadIdx.x / WAVE);
}

// A block's items left to a chain search go one per thread when at least this many are
// left (and the chains are monotone), else one at a time to a wavefront: a thread's
// bisections and edge run take several times a wavefront's latency for one item, but run
// side by side.
constexpr int THREAD_ITEMS = 32;

// Stage K of level job lev (0: vertex classes, 1: face intervals, 2: volume fractions; each
// needs the previous one), block lb of the job's nb: one thread per item.  Items the quick
// tests leave open on a many-sided polygon are finished with the polygon staged in LDS:
// vertex classes a tile of vertices per wavefront (geo_vertex_tile), faces and cells by
// chain search (THREAD_ITEMS).  The whole block calls it.
// The job's items are taken nb T_WIDE at a time (the launch grid is capped, so a large
// region takes several passes).
// MB: a context with several bodies (posed by the host; one thread per item).
template <int K, bool MB = false>
__device__ __forceinline__ void geo_stage_block(const StepArgs& a, int lev, int lb, int nb, double* spoly) {
    const GeoJob& J = a.geo[lev];
    if (!J.active) return;
    if (MB) {
        geo_bodies_block<K>(a.g, J, lb, nb, a.status);
        return;
    }
    // the vertex stage also poses the polygon: every block poses its own copy in LDS (the
    // level's copy is written in this launch, by the first block, for the later stages)
    Poly P = J.L.poly;
    bool staged = false;
    int mono = -1;  // the chains are monotone: 1, not: 0, not checked: -1
    if (K == 0) {
        if (lb == 0)
            for (int k = threadIdx.x; k < J.L.poly.m; k += blockDim.x) geo_pose(J, k);
        P = pose_lds(J, spoly);
        staged = true;
        if (P.m > SMALL_POLY) {
            __shared__ __attribute__((aligned(16))) unsigned short unc[T_WIDE / WAVE][UNC_CAP];
            int wv = threadIdx.x / WAVE, nwv = blockDim.x / WAVE;
            int tiles = geo_vertex_tiles(J.reg);
            for (int q = lb * nwv + wv; q < tiles; q += nb * nwv)
                geo_vertex_tile(a.g, J, P, q, unc[wv], threadIdx.x & (WAVE - 1));
            __syncthreads();  // the staged polygon may be overwritten next
            return;
        }
    }
    int items = K == 0 ? geo_nverts(J.reg) : (K == 1 ? geo_nfaces(J.reg) : J.reg.w() * J.reg.h());
    for (int base = 0; base < items; base += nb * T_WIDE) {
        int t = spread_item(lb, nb) + base;
        bool need = K == 0 ? geo_vertices1(a.g, J, P, t) : (K == 1 ? geo_faces1(a.g, J, t) : geo_cells1(a.g, J, t));
        int nneed = __syncthreads_count(need);
        if (nneed == 0) continue;
        if (!staged) {
            P = stage_poly(J.L.poly, spoly);
            staged = true;
        }
        Poly Pl = P;
        Pl.v = spoly;  // the staged copy (known to be in LDS)
        if (nneed >= THREAD_ITEMS && mono < 0) mono = chains_monotone(Pl);  // checked once, when needed
        if (mono > 0 && nneed >= THREAD_ITEMS) {
            each_left(need, t, [&](int item) {
                if (K == 1) geo_face_thread(a.g, J, Pl, item);
                if (K == 2) geo_cell_thread(a.g, J, Pl, item);
            });
            continue;
        }
        walk_left(need, t, [&](int item, int lane) {
            if (K == 0) geo_vertex_walk(a.g, J, Pl, item, lane);
            if (K == 1) geo_face_chain(a.g, J, Pl, item, lane);
            if (K == 2) geo_cell_chain(a.g, J, Pl, item, lane);
        });
    }
    __syncthreads();  // the staged polygon may be overwritten next
}

// Stage K of both level jobs of a member: the first half of its nb blocks works on level
// job 0, the second half on job 1 (the whole block calls it).
template <int K, bool MB = false>
__device__ __forceinline__ void geo_stage_split(const StepArgs& a, int lb, int nb, double* spoly) {
    int half = nb >> 1;
    int lev = lb >= half ? 1 : 0;
    geo_stage_block<K, MB>(a, lev, lb - lev * half, half, spoly);
}

// Stage K of both level jobs of every member.
template <int K, bool MB = false>
__global__ __launch_bounds__(T_WIDE) void kb_geo(const StepArgs* __restrict__ A, const int* __restrict__ off, int n) {
    __shared__ __attribute__((aligned(16))) double spoly[2 * LDS_VERTS];
    Unit w = unit_of(off, n);
    geo_stage_split<K, MB>(A[w.u], w.lb, w.nb, spoly);
}

// ------------------------------------------------------------------ sweeps
__device__ __forceinline__ bool box_empty_dev(const Box& B) { return B.i0 >= B.i1 || B.j0 >= B.j1; }

template <bool MB = false>
__device__ __forceinline__ void swept_block(const StepArgs& a, int s, int lb, int nb, double* spoly);

// Time-averaged apertures of sweep s over the faces of block lb (of nb) of the sweep box;
// faces left open by the quick tests on a many-sided polygon by chain search (THREAD_ITEMS).
template <bool MB>
__device__ __forceinline__ void swept_block(const StepArgs& a, int s, int lb, int nb, double* spoly) {
    const SweepJob& J = a.sw[s];
    if (box_empty_dev(J.B)) return;
    Stage S = stage_of(a, s);
    int items = J.dir == 0 ? (J.B.w() + 1) * J.B.h() : J.B.w() * (J.B.h() + 1);
    if (MB) {  // several bodies
        for (int t = lb * T_WIDE + (int)threadIdx.x; t < items; t += nb * T_WIDE) {
            if (J.dir == 0) swept_bodies<0>(a.g, J, a.bmot, S, t);
            else swept_bodies<1>(a.g, J, a.bmot, S, t);
        }
        return;
    }
    bool staged = false;
    int mono = -1;
    Poly P = J.Ls.poly;
    for (int base = 0; base < items; base += nb * T_WIDE) {  // the grid is capped: several passes
        int t = spread_item(lb, nb) + base;
        bool need = J.dir == 0 ? swept1<0>(a.g, J, a.mot, S, t) : swept1<1>(a.g, J, a.mot, S, t);
        int nneed = __syncthreads_count(need);
        if (nneed == 0) continue;
        if (!staged) {
            P = stage_poly(J.Ls.poly, spoly);
            staged = true;
        }
        Poly Pl = P;
        Pl.v = spoly;  // the staged copy (known to be in LDS)
        if (nneed >= THREAD_ITEMS && mono < 0) mono = chains_monotone(Pl);  // checked once, when needed
        if (mono > 0 && nneed >= THREAD_ITEMS) {
            each_left(need, t, [&](int item) {
                if (J.dir == 0) swept_thread<0>(a.g, J, Pl, a.mot, S, item);
                else swept_thread<1>(a.g, J, Pl, a.mot, S, item);
            });
            continue;
        }
        walk_left(need, t, [&](int item, int lane) {
            if (J.dir == 0) swept_chain<0>(a.g, J, Pl, a.mot, S, item, lane);
            else swept_chain<1>(a.g, J, Pl, a.mot, S, item, lane);
        });
    }
    __syncthreads();  // the staged polygon may be overwritten next
}

template <bool MB = false>
__global__ __launch_bounds__(T_WIDE) void kb_swept(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                   int n, int s) {
    __shared__ __attribute__((aligned(16))) double spoly[2 * LDS_VERTS];
    Unit w = unit_of(off, n);
    swept_block<MB>(A[w.u], s, w.lb, w.nb, spoly);
}

// Volume fractions of both level jobs and the time-averaged apertures of both sweeps (they
// need only the face intervals of the three levels) in one launch: a member's first
// nb_cells blocks do the cells, the next nb_swept the first sweep's faces, the last
// nb_swept the second sweep's.
template <bool MB = false>
__global__ __launch_bounds__(T_WIDE) void kb_geo_cells_swept(const StepArgs* __restrict__ A,
                                                             const int* __restrict__ off, int n) {
    __shared__ __attribute__((aligned(16))) double spoly[2 * LDS_VERTS];
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    int lb = w.lb;
    if (lb < a.nb_cells) {
        geo_stage_split<2, MB>(a, lb, a.nb_cells, spoly);
        return;
    }
    lb -= a.nb_cells;
    int s = lb >= a.nb_swept ? 1 : 0;
    swept_block<MB>(a, s, lb - s * a.nb_swept, a.nb_swept, spoly);
}

template <typename R, bool MB = false>
__device__ __forceinline__ void stagewall_body(const StepArgs& a, int s, int t) {
    const SweepJob& J = a.sw[s];
    if (t == 0) a.S.nbad[0] = a.S.nbad[1] = 0u;  // counters read later in this sweep
    if (box_empty_dev(J.B)) return;
    Stage S = stage_of(a, s);
    if (J.dir == 0) stagewall<0, R, MB>(a.g, J, a.mot, S, a.C, a.status, a.step_id, t, a.bmot);
    else stagewall<1, R, MB>(a.g, J, a.mot, S, a.C, a.status, a.step_id, t, a.bmot);
}

// Box cells t, t + stride, ... of sweep s (the launch grid is capped; at least the first
// call runs, which clears the sweep's counters).
// Axisymmetric form (the Euler equations of the shock tube of Sec. 3.5 in (x, r), r = y):
// the geometric source -(1/r) (rho v, rho u v, rho v^2, v (E + p)) as an operator step of
// length dt before the step's first sweep, on the content per cell volume (the source is
// homogeneous of degree one in the state, so S(U) = alpha S(Q)), r the cell centre's radius;
// cells without content are skipped.  One instance (its first sweep's input, updated in
// place).
template <typename R>
__global__ __launch_bounds__(256) void k_axisym(const StepArgs* __restrict__ A) {
    const StepArgs& a = A[0];
    const Grid& g = a.g;
    R* U = (R*)a.sw[0].Uin;
    size_t nc = (size_t)g.nx * g.ny;
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < nc; k += (size_t)gridDim.x * 256) {
        int j = (int)(k / (size_t)g.nx);
        double r = vy_of(g, j) + 0.5 * g.hy;
        double f = a.dt / r;
        double rho = (double)U[k], mx = (double)U[nc + k], my = (double)U[2 * nc + k], e = (double)U[3 * nc + k];
        if (!(rho > 0.0)) continue;
        double v = my / rho;
        double p = (g.gamma - 1.0) * (e - 0.5 * (mx * mx + my * my) / rho);
        U[k] = (R)(rho - f * my);
        U[nc + k] = (R)(mx - f * (mx * v));
        U[2 * nc + k] = (R)(my - f * (my * v));
        U[3 * nc + k] = (R)(e - f * (v * (e + p)));
    }
}

template <typename R, bool MB = false>
__device__ __forceinline__ void stagewall_loop(const StepArgs& a, int s, int t, int stride) {
    const SweepJob& J = a.sw[s];
    int cells = box_empty_dev(J.B) ? 0 : J.B.w() * J.B.h();
    do {
        stagewall_body<R, MB>(a, s, t);
        t += stride;
    } while (t < cells);
}

// MB: a context with several bodies (its box phase always has this launch of its own).
template <typename R, bool MB = false>
__global__ __launch_bounds__(T_BOX) void kb_stagewall(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                      int n, int s) {
    Unit w = unit_of(off, n);
    stagewall_loop<R, MB>(A[w.u], s, w.lb * T_BOX + threadIdx.x, w.nb * T_BOX);
}


// The patch update by line segments of the sweep direction (block lb of the member's
// patch_line_blocks<D>); the x sweep's patch runs it, the y sweep's runs the tiles below.
// One kernel per direction (members whose sweep runs the other way return at once): the
// update is the largest body, and one direction per kernel keeps it in registers.
template <int D, typename R>
__global__ __launch_bounds__(PL_T) void kb_patch_lines(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                       int n, int s) {
    __shared__ PatchLds sh;
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    const SweepJob& J = a.sw[s];
    if (J.dir != D || box_empty_dev(J.B)) return;
    int len = D == 0 ? J.B.w() : J.B.h(), nlines = D == 0 ? J.B.h() : J.B.w();
    int total = nlines * ((len + PL_OUT - 1) / PL_OUT);
    for (int lb = w.lb; lb < total; lb += w.nb)  // the grid is capped: several segments per block
        patch_line<D, R>(a.g, J, stage_of(a, s), a.ncol, lb, sh, a.bs);
}

// The y sweep's patch update by tiles of adjacent columns (block lb of the member's
// patch_tile_blocks).
template <typename R>
__global__ __launch_bounds__(PT_T) void kb_patch_tiles(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                       int n, int s) {
    __shared__ TileLds sh;
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    const SweepJob& J = a.sw[s];
    if (J.dir != 1 || box_empty_dev(J.B)) return;
    int total = patch_tile_blocks(J.B.w(), J.B.h());
    for (int lb = w.lb; lb < total; lb += w.nb)  // the grid is capped: several tiles per block
        patch_tile_y<R>(a.g, J, stage_of(a, s), a.ncol, lb, sh, a.bs);
}

template <typename R>
__device__ __forceinline__ void box_speeds(const StepArgs& a, int s, int t);

// speeds: the sweep is the last of a captured step: the box cells' wave speeds (of the
// covered state; the collapse rounds recompute them if they move content) go to the box
// blocks' partial pairs.
template <typename R>
__global__ __launch_bounds__(T_BOX) void kb_cover(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                  int n, int s, int speeds) {
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    const SweepJob& J = a.sw[s];
    int cells = box_empty_dev(J.B) ? 0 : J.B.w() * J.B.h();
    // 64 cells (one wavefront, one partial slot) at a time; the grid is capped
    for (int base = w.lb * T_BOX; base < cells; base += w.nb * T_BOX) {
        int t = base + threadIdx.x;
        double lost[4] = {0.0, 0.0, 0.0, 0.0};
        cover<R>(a.g, J, a.S, t, lost, a.bs.base != nullptr);
        if (a.bs.base) {  // T_BOX is one wavefront
#pragma unroll
            for (int m = 0; m < 4; m++) {
                double v = wave_sum(lost[m]);
                if (threadIdx.x == 0) a.bs.base[a.bs.cover + 4 * (base >> 6) + m] = v;
            }
        }
        if (speeds) box_speeds<R>(a, s, t);  // reads back the thread's own cell
    }
}

// fold: 1 when the sweep is the last of a captured step: every tile also writes the
// maxima of its cells' speeds to its partial pair.
__device__ __forceinline__ unsigned long long* fold_target(const StepArgs& a, int fold) {
    return fold ? a.spd : nullptr;
}

// Dense tiles of sweep s, block b of the launch's dense part (the whole block calls it).
template <typename R, int RB>
__device__ __forceinline__ void dense_x_block(const StepArgs* __restrict__ A, const int* __restrict__ off, int n,
                                              int b, int s, int fold, R* lds) {
    Unit w = unit_at(off, n, b);
    const StepArgs& a = A[w.u];
    const SweepJob& J = a.sw[s];
    if (J.dir != 0 || w.lb >= dense_x_blocks<RB>(a.g.nx, a.g.ny)) return;
    unsigned long long* cfl = fold_target(a, fold);
    dense_x<R, R, RB>(a.g, (const R*)J.Uin, (R*)J.Uout, J.B, (R)J.lam, w.lb, lds, cfl, a.bs.base);
}
template <typename R, int TR>
__device__ __forceinline__ void dense_y_block(const StepArgs* __restrict__ A, const int* __restrict__ off, int n,
                                              int b, int s, int fold, R* lds) {
    Unit w = unit_at(off, n, b);
    const StepArgs& a = A[w.u];
    const SweepJob& J = a.sw[s];
    if (J.dir != 1 || w.lb >= dense_y_blocks<TR>(a.g.nx, a.g.ny)) return;
    unsigned long long* cfl = fold_target(a, fold);
    dense_y<R, R, TR>(a.g, (const R*)J.Uin, (R*)J.Uout, J.B, (R)J.lam, w.lb, lds, cfl, a.bs.base);
}

template <typename R, int RW>
__device__ __forceinline__ void dense_yc_block(const StepArgs* __restrict__ A, const int* __restrict__ off, int n,
                                               int b, int s, int fold) {
    Unit w = unit_at(off, n, b);
    const StepArgs& a = A[w.u];
    const SweepJob& J = a.sw[s];
    if (J.dir != 1 || w.lb >= dense_yc_blocks<RW>(a.g.nx, a.g.ny)) return;
    unsigned long long* cfl = fold_target(a, fold);
    dense_yc<R, R, RW>(a.g, (const R*)J.Uin, (R*)J.Uout, J.B, (R)J.lam, w.lb, cfl, a.bs.base);
}

template <typename R, int RB>
__global__ __launch_bounds__(DX_T) void kb_dense_x(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                   int n, int s, int fold) {
    dense_x_block<R, RB>(A, off, n, blockIdx.x, s, fold, nullptr);
}

template <typename R, int TR>
__global__ __launch_bounds__(256) void kb_dense_y(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                  int n, int s, int fold) {
    __shared__ R lds[DenseYTile<R, TR>::lds_bytes / sizeof(R)];
    dense_y_block<R, TR>(A, off, n, blockIdx.x, s, fold, lds);
}

template <typename R, int RW>
__global__ __launch_bounds__(DYC_T) void kb_dense_yc(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                     int n, int s, int fold) {
    dense_yc_block<R, RW>(A, off, n, blockIdx.x, s, fold);
}

// The box cells' first phase of sweep s (donations and wall quantities) in the same launch
// as the dense tiles: the two touch disjoint data (the tiles read the state and write the
// cells outside the box; the box phase reads the state and geometry and writes box-local
// staging), so the box's latency-bound cells run while the tiles stream.  The first nwall
// blocks are box blocks (T_WIDE cells each, table off_wall), the rest dense blocks.
template <typename R, int RB>
__global__ __launch_bounds__(DX_T) __attribute__((amdgpu_waves_per_eu(4))) void kb_wall_dense_x(const StepArgs* __restrict__ A,
                                                        const int* __restrict__ off_wall, int nwall,
                                                        const int* __restrict__ off, int n, int s, int fold) {
    if ((int)blockIdx.x < nwall) {
        Unit w = unit_at(off_wall, n, blockIdx.x);
        stagewall_loop<R>(A[w.u], s, w.lb * T_WIDE + threadIdx.x, w.nb * T_WIDE);
        return;
    }
    dense_x_block<R, RB>(A, off, n, blockIdx.x - nwall, s, fold, nullptr);
}
template <typename R, int TR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void kb_wall_dense_y(const StepArgs* __restrict__ A,
                                                       const int* __restrict__ off_wall, int nwall,
                                                       const int* __restrict__ off, int n, int s, int fold) {
    __shared__ R lds[DenseYTile<R, TR>::lds_bytes / sizeof(R)];
    if ((int)blockIdx.x < nwall) {
        Unit w = unit_at(off_wall, n, blockIdx.x);
        stagewall_loop<R>(A[w.u], s, w.lb * T_WIDE + threadIdx.x, w.nb * T_WIDE);
        return;
    }
    dense_y_block<R, TR>(A, off, n, blockIdx.x - nwall, s, fold, lds);
}

template <typename R, int RW>
__global__ __launch_bounds__(DYC_T) __attribute__((amdgpu_waves_per_eu(4))) void kb_wall_dense_yc(
    const StepArgs* __restrict__ A, const int* __restrict__ off_wall, int nwall, const int* __restrict__ off, int n,
    int s, int fold) {
    if ((int)blockIdx.x < nwall) {
        Unit w = unit_at(off_wall, n, blockIdx.x);
        stagewall_loop<R>(A[w.u], s, w.lb * T_WIDE + threadIdx.x, w.nb * T_WIDE);
        return;
    }
    dense_yc_block<R, RW>(A, off, n, blockIdx.x - nwall, s, fold);
}

// Wave speeds of box cell t of the member's sweep s (end level, state as stored); the
// wavefront's maxima go to the member's partial pair of box block t / 64.  Every lane of
// the wavefront calls it.
template <typename R>
__device__ __forceinline__ void box_speeds(const StepArgs& a, int s, int t) {
    const SweepJob& J = a.sw[s];
    unsigned long long bx = 0ull, by = 0ull;
    int w = J.B.w(), h = J.B.h();
    if (w > 0 && h > 0 && t < w * h) {
        int i = J.B.i0 + t % w, j = J.B.j0 + t / w;
        size_t nc = (size_t)a.g.nx * a.g.ny, k = (size_t)j * a.g.nx + i;
        const R* U = (const R*)J.Uout;
        R u[4];
#pragma unroll
        for (int m = 0; m < 4; m++) u[m] = U[m * nc + k];
        speed_bits(u, J.Le.alpha[k], a.g.gamma, bx, by);
    }
    wave_max_pair(bx, by);
    if ((threadIdx.x & 63) == 0) {
        unsigned long long* out = a.spd + 2 * (a.spd_dense + (t >> 6));
        out[0] = bx;
        out[1] = by;
    }
}

// Member u's time-step maxima from its partial pairs (the dense tiles of the step's last
// sweep, then its box blocks) and the block's own pair (bx, by), and its status word and
// collapse count gathered for one read-back.  Every thread of the block calls it.
__device__ __forceinline__ void combine_speeds(const StepArgs& a, int ndense, int nbox, unsigned int* gather, int u,
                                               unsigned long long bx = 0ull, unsigned long long by = 0ull) {
    // the dense tiles used slot pairs 0 .. min(ndense, NSPD) - 1; each is read and reset to
    // zero by one thread, ready for the next step
    int nd = ndense < NSPD ? ndense : NSPD;
    for (int k = threadIdx.x; k < nd + nbox; k += blockDim.x) {
        int q = k < nd ? k : a.spd_dense + (k - nd);
        unsigned long long x = a.spd[2 * q], y = a.spd[2 * q + 1];
        if (k < nd) {
            a.spd[2 * q] = 0ull;
            a.spd[2 * q + 1] = 0ull;
        }
        bx = x > bx ? x : bx;
        by = y > by ? y : by;
    }
    __shared__ unsigned long long res[2];
    block_max_to(bx, by, res);
    if (threadIdx.x == 0) {
        a.cfl_out[0] = res[0];
        a.cfl_out[1] = res[1];
        gather[2 * u] = *a.status;
        gather[2 * u + 1] = *a.ncol;
    }
}

constexpr int T_FIX = 256;  // threads of the per-member collapse block

// Adds the sweep's budget to the member's running sums: the fluxes through the domain
// boundary (dense slots, then the patch blocks' end faces) times dt/h and the cell
// area, the wall terms likewise, and the residuals without recipients (covering blocks,
// then the collapse rounds' `lost` of each thread) times the cell area.  Each thread sums
// a fixed subset of the slots, then the block adds the threads' sums in a fixed tree, so
// the result does not depend on timing.  Every thread of the block calls it.
__device__ __forceinline__ void sweep_budget(const StepArgs& a, const SweepJob& J, int cells, const double* lost) {
    const double* bs = a.bs.base;
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; q++) acc[q] = 0.0;  // lo, hi, wall, lost (4 components each)
    int nd = (int)bs[0];
    for (int k = threadIdx.x; k < nd; k += blockDim.x) {
        int side = k & 1;
#pragma unroll
        for (int m = 0; m < 4; m++) acc[4 * side + m] += bs[BS_DENSE + 4 * k + m];
    }
    int np = 0, ncov = 0;
    if (cells > 0) {
        np = J.dir == 0 ? J.B.h() * ((J.B.w() + PL_OUT - 1) / PL_OUT) : patch_tile_blocks(J.B.w(), J.B.h());
        ncov = (cells + T_BOX - 1) / T_BOX;
    }
    for (int k = threadIdx.x; k < np; k += blockDim.x)
#pragma unroll
        for (int q = 0; q < 12; q++) acc[q] += bs[a.bs.patch + 12 * k + q];
    for (int k = threadIdx.x; k < ncov; k += blockDim.x)
#pragma unroll
        for (int m = 0; m < 4; m++) acc[12 + m] += bs[a.bs.cover + 4 * k + m];
#pragma unroll
    for (int m = 0; m < 4; m++) acc[12 + m] += lost[m];
    __shared__ double red[16][T_FIX / 64];
    int wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 16; q++) {
        double v = wave_sum(acc[q]);
        if ((threadIdx.x & 63) == 0) red[q][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[16];
        for (int q = 0; q < 16; q++) {
            tot[q] = red[q][0];
            for (int w = 1; w < (int)(blockDim.x >> 6); w++) tot[q] += red[q][w];
        }
        double area = a.g.hx * a.g.hy, f = J.lam * area;
        for (int m = 0; m < 4; m++) {
            a.budget[m] += f * (tot[m] - tot[4 + m]);
            a.budget[4 + m] += f * tot[8 + m];
            a.budget[8 + m] += area * tot[12 + m];
        }
    }
    __syncthreads();
}

// Both collapse rounds of sweep s (reading R28) for every member, one block per member:
// both return at once unless covering left a bad cell, which is rare, so one block walks
// the whole box, with a block barrier between the rounds.  last: the sweep is the last of
// a captured step; the block then also combines the member's wave-speed partials (the box
// cells' speeds recomputed here when a round moved content) and gathers its status words.
template <typename R>
__global__ __launch_bounds__(T_FIX) void kb_fix_block(StepArgs* A, const int* __restrict__ off_dx,
                                                      const int* __restrict__ off_dy,
                                                      const int* __restrict__ off_box, int s, int last,
                                                      unsigned int* __restrict__ gather) {
    int u = blockIdx.x;
    const StepArgs& a = A[u];
    const SweepJob& J = a.sw[s];
    int cells = box_empty_dev(J.B) ? 0 : J.B.w() * J.B.h();
    bool bad = cells > 0 && __hip_atomic_load(&a.S.nbad[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    double lost[4] = {0.0, 0.0, 0.0, 0.0};  // this thread's collapsed cells without recipients
    if (bad)
        for (int round = 0; round < 2; round++) {
            for (int t = threadIdx.x; t < cells; t += blockDim.x)
                fix<R>(a.g, J, a.S, round, a.ncol, a.status, t, lost, a.bs.base != nullptr);
            __syncthreads();  // the round's flags and contents, for the next round and the speeds
        }
    if (a.bs.base) sweep_budget(a, J, cells, lost);
    if (!last) return;
    unsigned long long bx = 0ull, by = 0ull;
    if (bad) {
        const R* U = (const R*)J.Uout;
        size_t nc = (size_t)a.g.nx * a.g.ny;
        for (int t = threadIdx.x; t < cells; t += blockDim.x) {
            int i = J.B.i0 + t % J.B.w(), j = J.B.j0 + t / J.B.w();
            size_t k = (size_t)j * a.g.nx + i;
            R uu[4];
#pragma unroll
            for (int m = 0; m < 4; m++) uu[m] = U[m * nc + k];
            unsigned long long cx, cy;
            speed_bits(uu, J.Le.alpha[k], a.g.gamma, cx, cy);
            bx = cx > bx ? cx : bx;
            by = cy > by ? cy : by;
        }
    }
    const int* od = a.sw[1].dir == 0 ? off_dx : off_dy;
    // with recomputed box speeds the box cells' partials (of the covered state) are skipped;
    // otherwise one pair per 64 box cells
    combine_speeds(a, od[u + 1] - od[u], bad ? 0 : (cells + T_BOX - 1) / T_BOX, gather, u, bx, by);
    (void)off_box;
    const PlanConst* pc = a.pc;
    PlanState* ps = a.ps;
    double* dl = a.dtlog;
    __syncthreads();  // the combined speeds are written; the step's arguments are read no more
    if (pc) plan_block(pc, ps, &A[u], dl);
}

}  // namespace cc
