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

namespace cc {

struct StepArgs {
    Grid g;
    GeoJob geo[2];   // stage level and end level of the step
    SweepJob sw[2];  // first and second sweep
    Motion mot;
    Stage S;
    Common C;
    unsigned int* status;
    unsigned int* ncol;
    double* bt[2];          // time-averaged apertures of each sweep (box-local faces)
    int* slist[2];          // work lists of the swept apertures left to phase 2, per sweep
    unsigned int* scnt[2];  // their lengths
    int32_t step_id;
    // time-step reduction of the state after the step
    const double* cfl_alpha;
    const void* cfl_U;
    unsigned long long* cfl_part;  // 2 per block
    unsigned long long* cfl_out;   // 2: max (|u|+a) along x and y, as bit patterns
    unsigned long long* spd;       // 2 x SPEED_SLOTS: the same maxima folded in by a captured step
};

// Launch kinds and their block sizes.
enum LaunchKind {
    L_POSE, L_V1, L_V2, L_F1, L_F2, L_C1, L_C2,  // geometry of one level
    L_S1, L_S2, L_BOX, L_DX, L_DY, L_CFL, L_CFLF,  // sweeps and time step
    L_BSPD,  // wave speeds of the box cells after the step (at least one block per member)
    NKINDS
};
constexpr int T_WIDE = 256;  // phase 1, phase 2 (4 wavefronts), dense, time step
constexpr int T_BOX = 64;    // box phases: a few thousand cells spread over all CUs
constexpr int ITEMS_PER_BLOCK = T_WIDE / WAVE;

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
__device__ __forceinline__ Unit unit_of(const int* __restrict__ off, int n) {
    Unit r;
    r.u = n == 1 ? 0 : find_unit(off, n, blockIdx.x);
    r.lb = blockIdx.x - off[r.u];
    r.nb = off[r.u + 1] - off[r.u];
    return r;
}

// ------------------------------------------------------------------ geometry
// Geometry launches work on one level job (lev) of every member.
// Level job lev: pose the polygon; the first thread also clears the job's phase-2 list
// lengths (and, for the first job, those of both sweeps' aperture lists).
__device__ __forceinline__ void pose_body(const StepArgs& a, int lev, int t) {
    const GeoJob& J = a.geo[lev];
    if (t == 0 && lev == 0) *a.scnt[0] = *a.scnt[1] = 0u;
    if (!J.active) return;
    if (t == 0) J.cnt[0] = J.cnt[1] = J.cnt[2] = 0u;
    geo_pose(J, t);
}

__global__ __launch_bounds__(T_WIDE) void kb_geo_pose(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                      int n, int lev) {
    Unit w = unit_of(off, n);
    pose_body(A[w.u], lev, w.lb * T_WIDE + threadIdx.x);
}

// Stage arrays of sweep s (the apertures are per sweep, the rest is shared).
__device__ __forceinline__ Stage stage_of(const StepArgs& a, int s) {
    Stage S = a.S;
    S.bt = a.bt[s];
    return S;
}

template <int K>
__global__ __launch_bounds__(T_WIDE) void kb_geo_p1(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                    int n, int lev) {
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    const GeoJob& J = a.geo[lev];
    if (!J.active) return;
    int t = w.lb * T_WIDE + threadIdx.x;
    bool need;
    if (K == 0) need = geo_vertices1(a.g, J, t);
    if (K == 1) need = geo_faces1(a.g, J, t);
    if (K == 2) need = geo_cells1(a.g, J, t);
    list_append(J.list, &J.cnt[K], need, t);
}

// The polygon of a phase-2 block, staged in LDS when it fits (every wavefront of the block
// walks all its edges for each of its items).
constexpr int LDS_VERTS = 2048;
constexpr size_t POLY_LDS = (size_t)2 * LDS_VERTS * sizeof(double);
__device__ __forceinline__ Poly stage_poly(const Poly& P, double* spoly) {
    Poly Q = P;
    if (P.m <= LDS_VERTS) {
        for (int k = threadIdx.x; k < 2 * P.m; k += blockDim.x) spoly[k] = P.v[k];
        __syncthreads();
        Q.v = spoly;
    }
    return Q;
}

// Phase-2 items of virtual block lb (of nb) of a level job: one wavefront per item, the
// polygon staged in LDS.  Every thread of the block calls it (it synchronises the block).
template <int K>
__device__ __forceinline__ void geo_p2_block(const StepArgs& a, int lev, int lb, int nb, double* spoly) {
    const GeoJob& J = a.geo[lev];
    if (!J.active) return;
    int items = (int)J.cnt[K];
    if (lb * ITEMS_PER_BLOCK >= items) return;  // no item for this block
    Poly P = stage_poly(J.L.poly, spoly);
    int lane = threadIdx.x & (WAVE - 1);
    for (int it = lb * ITEMS_PER_BLOCK + (threadIdx.x >> 6); it < items; it += nb * ITEMS_PER_BLOCK) {
        if (K == 0) geo_vertices2(a.g, J, P, it, lane);
        if (K == 1) geo_faces2(a.g, J, P, it, lane);
        if (K == 2) geo_cells2(a.g, J, P, it, lane);
    }
    __syncthreads();  // the staged polygon may be overwritten next
}

template <int K>
__global__ __launch_bounds__(T_WIDE) void kb_geo_p2(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                    int n, int lev) {
    __shared__ double spoly[2 * LDS_VERTS];
    Unit w = unit_of(off, n);
    geo_p2_block<K>(A[w.u], lev, w.lb, w.nb, spoly);
}

// ------------------------------------------------------------------ sweeps
__device__ __forceinline__ bool box_empty_dev(const Box& B) { return B.i0 >= B.i1 || B.j0 >= B.j1; }

// Swept apertures of sweep s, phase 1 (thread t of the member).
__device__ __forceinline__ void swept1_body(const StepArgs& a, int s, int t) {
    const SweepJob& J = a.sw[s];
    if (box_empty_dev(J.B)) return;
    Stage S = stage_of(a, s);
    bool need = J.dir == 0 ? swept1<0>(a.g, J, a.mot, S, t) : swept1<1>(a.g, J, a.mot, S, t);
    list_append(a.slist[s], a.scnt[s], need, t);
}

// Swept apertures of sweep s, phase 2 (virtual block lb of nb; the whole block calls it).
__device__ __forceinline__ void swept2_block(const StepArgs& a, int s, int lb, int nb, double* spoly) {
    const SweepJob& J = a.sw[s];
    if (box_empty_dev(J.B)) return;
    int items = (int)*a.scnt[s];
    if (lb * ITEMS_PER_BLOCK >= items) return;  // no item for this block
    Stage S = stage_of(a, s);
    Poly P = stage_poly(J.Ls.poly, spoly);
    int lane = threadIdx.x & (WAVE - 1);
    for (int it = lb * ITEMS_PER_BLOCK + (threadIdx.x >> 6); it < items; it += nb * ITEMS_PER_BLOCK) {
        if (J.dir == 0) swept2<0>(a.g, J, P, a.mot, S, a.slist[s], it, lane);
        else swept2<1>(a.g, J, P, a.mot, S, a.slist[s], it, lane);
    }
    __syncthreads();  // the staged polygon may be overwritten next
}

__global__ __launch_bounds__(T_WIDE) void kb_swept1(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                    int n, int s) {
    Unit w = unit_of(off, n);
    swept1_body(A[w.u], s, w.lb * T_WIDE + threadIdx.x);
}

__global__ __launch_bounds__(T_WIDE) void kb_swept2(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                    int n, int s) {
    __shared__ double spoly[2 * LDS_VERTS];
    Unit w = unit_of(off, n);
    swept2_block(A[w.u], s, w.lb, w.nb, spoly);
}

template <typename R>
__device__ __forceinline__ void stagewall_body(const StepArgs& a, int s, int t) {
    const SweepJob& J = a.sw[s];
    if (t == 0) a.S.nbad[0] = a.S.nbad[1] = 0u;  // counters read later in this sweep
    if (box_empty_dev(J.B)) return;
    Stage S = stage_of(a, s);
    if (J.dir == 0) stagewall<0, R>(a.g, J, a.mot, S, a.C, a.status, a.step_id, t);
    else stagewall<1, R>(a.g, J, a.mot, S, a.C, a.status, a.step_id, t);
}

template <typename R>
__global__ __launch_bounds__(T_BOX) void kb_stagewall(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                      int n, int s) {
    Unit w = unit_of(off, n);
    stagewall_body<R>(A[w.u], s, w.lb * T_BOX + threadIdx.x);
}

// One kernel per direction (members whose sweep runs the other way return at once): the
// update is the largest body, and one direction per kernel keeps it in registers.
template <int D, typename R>
__global__ __launch_bounds__(T_BOX) void kb_patch(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                  int n, int s) {
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    const SweepJob& J = a.sw[s];
    if (J.dir != D || box_empty_dev(J.B)) return;
    patch<D, R>(a.g, J, stage_of(a, s), a.ncol, w.lb * T_BOX + threadIdx.x);
}

template <typename R>
__global__ __launch_bounds__(T_BOX) void kb_cover(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                  int n, int s) {
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    const SweepJob& J = a.sw[s];
    if (box_empty_dev(J.B)) return;
    cover<R>(a.g, J, a.S, w.lb * T_BOX + threadIdx.x);
}

template <typename R>
__global__ __launch_bounds__(T_BOX) void kb_fix(const StepArgs* __restrict__ A, const int* __restrict__ off, int n,
                                                int s, int round) {
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    const SweepJob& J = a.sw[s];
    if (box_empty_dev(J.B)) return;
    fix<R>(a.g, J, a.S, round, a.ncol, a.status, w.lb * T_BOX + threadIdx.x);
}

// fold: 0 plain sweep; 1 also clears the member's speed slots (first sweep of a captured
// step); 2 folds the speeds of the written cells into them (second sweep).
__device__ __forceinline__ void clear_speeds(const StepArgs& a) {
    for (int k = threadIdx.x; k < 2 * SPEED_SLOTS; k += blockDim.x) a.spd[k] = 0ull;
}
__device__ __forceinline__ unsigned long long* fold_target(const StepArgs& a, int lb, int fold) {
    if (fold == 1 && lb == 0) clear_speeds(a);
    return fold == 2 ? a.spd : nullptr;
}

template <typename R, int RB>
__global__ __launch_bounds__(DX_T) void kb_dense_x(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                   int n, int s, int fold) {
    __shared__ R lds[dense_x_lds<R>() / sizeof(R)];
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    const SweepJob& J = a.sw[s];
    if (J.dir != 0 || w.lb >= dense_x_blocks<RB>(a.g.nx, a.g.ny)) return;
    unsigned long long* cfl = fold_target(a, w.lb, fold);
    dense_x<R, R, RB>(a.g, (const R*)J.Uin, (R*)J.Uout, J.B, (R)J.lam, w.lb, lds, cfl);
}

template <typename R, int TR>
__global__ __launch_bounds__(256) void kb_dense_y(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                  int n, int s, int fold) {
    __shared__ R lds[DenseYTile<R, TR>::lds_bytes / sizeof(R)];
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    const SweepJob& J = a.sw[s];
    if (J.dir != 1 || w.lb >= dense_y_blocks<TR>(a.g.nx, a.g.ny)) return;
    unsigned long long* cfl = fold_target(a, w.lb, fold);
    dense_y<R, R, TR>(a.g, (const R*)J.Uin, (R*)J.Uout, J.B, (R)J.lam, w.lb, lds, cfl);
}

// Wave speeds of box cell t of the member's sweep s (end level, state as stored), folded
// into its time-step maxima.  Every lane of the wavefront calls it.
template <typename R>
__device__ __forceinline__ void box_speeds(const StepArgs& a, int s, int t) {
    const SweepJob& J = a.sw[s];
    unsigned long long bx = 0ull, by = 0ull;
    int w = J.B.w(), h = J.B.h();
    if (w > 0 && h > 0 && t < w * h) {
        int i = J.B.i0 + t % w, j = J.B.j0 + t / w;
        size_t nc = (size_t)a.g.nx * a.g.ny, k = (size_t)j * a.g.nx + i;
        const R* U = (const R*)J.Uout;
        double al = J.Le.alpha[k];
        double r = (double)U[k];
        if (al > 0.0 && r > 0.0) {
            double q[4];
#pragma unroll
            for (int m = 0; m < 4; m++) q[m] = (double)U[m * nc + k] / al;
            double uu = q[1] / q[0], vv = q[2] / q[0];
            double c = sqrt(a.g.gamma * pressure(q, a.g.gamma) / q[0]);
            double sx = fabs(uu) + c, sy = fabs(vv) + c;
            bx = __double_as_longlong(sx);
            by = __double_as_longlong(sy);
            if (sx != sx) bx = 0x7ff8000000000000ull;
            if (sy != sy) by = 0x7ff8000000000000ull;
        }
    }
    speeds_to_max(bx, by, a.spd);
}

// After the second sweep of a captured step: the box cells' wave speeds (the host takes
// the maximum over the speed slots it reads back), and the status word and collapse count
// of each member gathered for the same read-back.
template <typename R>
__global__ __launch_bounds__(T_BOX) void kb_box_speeds(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                       int n, unsigned int* __restrict__ gather) {
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    box_speeds<R>(a, 1, w.lb * T_BOX + threadIdx.x);
    if (w.lb == 0 && threadIdx.x == 0) {
        gather[2 * w.u] = *a.status;
        gather[2 * w.u + 1] = *a.ncol;
    }
}

// ------------------------------------------------------------------ time step
// Per-block maxima of |u|+a along x and y over the live cells of each instance (bit
// patterns of non-negative doubles order like the values; NaN sorts above infinity), then
// one block per instance combines its partials.
template <typename R>
__global__ __launch_bounds__(T_WIDE) void kb_cfl(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                 int n) {
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    cfl_block<R>(a.g, a.cfl_alpha, (const R*)a.cfl_U, a.cfl_part, w.lb, w.nb);
}

__global__ __launch_bounds__(T_WIDE) void kb_cfl_final(const StepArgs* __restrict__ A,
                                                       const int* __restrict__ off_cfl, int n) {
    const StepArgs& a = A[blockIdx.x];
    int nparts = off_cfl[blockIdx.x + 1] - off_cfl[blockIdx.x];
    cfl_combine(nparts, a.cfl_part, a.cfl_out);
}

// Status word and collapse count of every instance, gathered for one read-back.
__global__ void kb_gather(const StepArgs* __restrict__ A, int n, unsigned int* __restrict__ out) {
    int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    out[2 * u] = *A[u].status;
    out[2 * u + 1] = *A[u].ncol;
}

}  // namespace cc
