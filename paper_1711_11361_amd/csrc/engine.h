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
    int* slist;  // work list of the swept apertures left to phase 2
    unsigned int* scnt;
    int32_t step_id;
    // time-step reduction of the state after the step
    const double* cfl_alpha;
    const void* cfl_U;
    unsigned long long* cfl_part;  // 2 per block
    unsigned long long* cfl_out;   // 2: max (|u|+a) along x and y, as bit patterns
};

// Launch kinds and their block sizes.
enum LaunchKind {
    L_POSE, L_V1, L_V2, L_F1, L_F2, L_C1, L_C2,  // geometry of one level
    L_S1, L_S2, L_BOX, L_DX, L_DY, L_CFL, L_CFLF,  // sweeps and time step
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
    r.u = find_unit(off, n, blockIdx.x);
    r.lb = blockIdx.x - off[r.u];
    r.nb = off[r.u + 1] - off[r.u];
    return r;
}

// ------------------------------------------------------------------ geometry
// Geometry launches work on one level job (lev) of every member.
__global__ __launch_bounds__(T_WIDE) void kb_geo_pose(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                      int n, int lev) {
    Unit w = unit_of(off, n);
    const GeoJob& J = A[w.u].geo[lev];
    if (!J.active) return;
    int t = w.lb * T_WIDE + threadIdx.x;
    if (t == 0) J.cnt[0] = J.cnt[1] = J.cnt[2] = 0u;  // lists of this level's phases
    geo_pose(J, t);
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
__device__ __forceinline__ Poly stage_poly(const Poly& P, double* spoly) {
    Poly Q = P;
    if (P.m <= LDS_VERTS) {
        for (int k = threadIdx.x; k < 2 * P.m; k += blockDim.x) spoly[k] = P.v[k];
        __syncthreads();
        Q.v = spoly;
    }
    return Q;
}

template <int K>
__global__ __launch_bounds__(T_WIDE) void kb_geo_p2(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                    int n, int lev) {
    __shared__ double spoly[2 * LDS_VERTS];
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    const GeoJob& J = a.geo[lev];
    if (!J.active) return;
    int items = (int)J.cnt[K];
    if (w.lb * ITEMS_PER_BLOCK >= items) return;  // no item for this block
    Poly P = stage_poly(J.L.poly, spoly);
    int lane = threadIdx.x & (WAVE - 1);
    for (int it = w.lb * ITEMS_PER_BLOCK + (threadIdx.x >> 6); it < items; it += w.nb * ITEMS_PER_BLOCK) {
        if (K == 0) geo_vertices2(a.g, J, P, it, lane);
        if (K == 1) geo_faces2(a.g, J, P, it, lane);
        if (K == 2) geo_cells2(a.g, J, P, it, lane);
    }
}

// ------------------------------------------------------------------ sweeps
__device__ __forceinline__ bool box_empty_dev(const Box& B) { return B.i0 >= B.i1 || B.j0 >= B.j1; }

__global__ __launch_bounds__(T_WIDE) void kb_swept1(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                    int n, int s) {
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    const SweepJob& J = a.sw[s];
    if (box_empty_dev(J.B)) return;
    int t = w.lb * T_WIDE + threadIdx.x;
    bool need = J.dir == 0 ? swept1<0>(a.g, J, a.mot, a.S, t) : swept1<1>(a.g, J, a.mot, a.S, t);
    list_append(a.slist, a.scnt, need, t);
}

__global__ __launch_bounds__(T_WIDE) void kb_swept2(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                    int n, int s) {
    __shared__ double spoly[2 * LDS_VERTS];
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    const SweepJob& J = a.sw[s];
    if (box_empty_dev(J.B)) return;
    int items = (int)*a.scnt;
    if (w.lb * ITEMS_PER_BLOCK >= items) return;  // no item for this block
    Poly P = stage_poly(J.Ls.poly, spoly);
    int lane = threadIdx.x & (WAVE - 1);
    for (int it = w.lb * ITEMS_PER_BLOCK + (threadIdx.x >> 6); it < items; it += w.nb * ITEMS_PER_BLOCK) {
        if (J.dir == 0) swept2<0>(a.g, J, P, a.mot, a.S, a.slist, it, lane);
        else swept2<1>(a.g, J, P, a.mot, a.S, a.slist, it, lane);
    }
}

template <typename R>
__global__ __launch_bounds__(T_BOX) void kb_stagewall(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                      int n, int s) {
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    const SweepJob& J = a.sw[s];
    int t = w.lb * T_BOX + threadIdx.x;
    if (t == 0) {  // counters read later in this sweep, or by the next sweep's apertures
        a.S.nbad[0] = a.S.nbad[1] = 0u;
        *a.scnt = 0u;
    }
    if (box_empty_dev(J.B)) return;
    if (J.dir == 0) stagewall<0, R>(a.g, J, a.mot, a.S, a.C, a.status, a.step_id, t);
    else stagewall<1, R>(a.g, J, a.mot, a.S, a.C, a.status, a.step_id, t);
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
    patch<D, R>(a.g, J, a.S, a.ncol, w.lb * T_BOX + threadIdx.x);
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

template <typename R, int RB>
__global__ __launch_bounds__(DX_T) void kb_dense_x(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                   int n, int s) {
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    const SweepJob& J = a.sw[s];
    if (J.dir != 0 || w.lb >= dense_x_blocks<RB>(a.g.nx, a.g.ny)) return;
    dense_x<R, R, RB>(a.g, (const R*)J.Uin, (R*)J.Uout, J.B, (R)J.lam, w.lb);
}

template <typename R, int TR>
__global__ __launch_bounds__(256) void kb_dense_y(const StepArgs* __restrict__ A, const int* __restrict__ off,
                                                  int n, int s) {
    Unit w = unit_of(off, n);
    const StepArgs& a = A[w.u];
    const SweepJob& J = a.sw[s];
    if (J.dir != 1 || w.lb >= dense_y_blocks<TR>(a.g.nx, a.g.ny)) return;
    dense_y<R, R, TR>(a.g, (const R*)J.Uin, (R*)J.Uout, J.B, (R)J.lam, w.lb);
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
