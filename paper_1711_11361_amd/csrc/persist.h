// One persistent launch per sweep over every member of a batch.  The launch's blocks are all
// resident at once (the host sizes the grid from the kernel's occupancy), so the phases of
// a sweep are separated by grid-wide barriers instead of kernel boundaries:
//   sweep 0: pose both level jobs | vertex classes | face intervals | volume fractions and
//            the swept apertures of both sweeps | stage and wall | patch | cover | collapse
//            round 1 | collapse round 2
//   sweep 1: stage and wall | patch | cover | collapse rounds | wave speeds of the box cells
// Each barrier has its own arrival counter.  Only the leading blocks that have work in the
// next phase wait at a barrier; every other block arrives and moves on.  The dense tiles of
// the sweep (every regular cell outside the sweep boxes) are independent of all phases:
// blocks take them from a queue once they have no phase work left, so the streaming update
// overlaps the chain of cut-cell phases.  In the second sweep the dense tiles and the last
// phase also fold the wave speeds of the new state into the members' time-step maxima, and
// the block that finishes last gathers the status words.
//
// A barrier wait is bounded: after a fixed wall-clock time the waiting block flags an
// error and goes on, so a launch always ends (the host reports the flag as a device error).
#pragma once
#include "engine.h"

namespace cc {

constexpr int MAX_BARRIERS = 16;
struct GridSync {
    unsigned int arrived[2][MAX_BARRIERS];  // arrivals per barrier of the sweep-0 / sweep-1 launch
    unsigned int queue[2];  // next dense tile of sweep 0 / 1
    unsigned int done;      // blocks that finished the current launch
    unsigned int err;       // 1: a barrier wait timed out
};  // all counters return to zero at the end of every launch (its last block resets them)

struct PArgs {
    const StepArgs* A;
    const int* off;  // launch tables, NKINDS x stride
    int n, stride;
    GridSync* gs;
    unsigned int* gather;  // 2 words per member (status, collapses), written after sweep 1
    unsigned long long wait_ticks;  // barrier time limit in wall-clock ticks
    int s;  // sweep 0 or 1
};

template <typename R, int TR>
__host__ __device__ constexpr size_t persist_lds() {
    size_t a = POLY_LDS, b = dense_x_lds<R>(), c = DenseYTile<R, TR>::lds_bytes;
    size_t m = a > b ? a : b;
    return m > c ? m : c;
}

__device__ __forceinline__ const int* ptab(const PArgs& p, int kind) { return p.off + (size_t)kind * p.stride; }

// Dense tile `tile` of the sweep: x tiles of every member, then y tiles; a member's tiles of
// the direction it does not sweep in are empty.  The whole block calls it.
template <typename R, int RB, int TR>
__device__ void dense_tile(const PArgs& p, unsigned int tile, unsigned char* lds) {
    const int* ox = ptab(p, L_DX);
    unsigned int tx = (unsigned int)ox[p.n];
    if (tile < tx) {
        int u = find_unit(ox, p.n, (int)tile);
        const StepArgs& a = p.A[u];
        const SweepJob& J = a.sw[p.s];
        int lb = (int)tile - ox[u];
        if (J.dir == 0 && lb < dense_x_blocks<RB>(a.g.nx, a.g.ny))
            dense_x<R, R, RB>(a.g, (const R*)J.Uin, (R*)J.Uout, J.B, (R)J.lam, lb, (R*)lds,
                              p.s == 1 ? a.spd : nullptr);
        return;
    }
    const int* oy = ptab(p, L_DY);
    int t = (int)(tile - tx);
    int u = find_unit(oy, p.n, t);
    const StepArgs& a = p.A[u];
    const SweepJob& J = a.sw[p.s];
    int lb = t - oy[u];
    if (J.dir == 1 && lb < dense_y_blocks<TR>(a.g.nx, a.g.ny))
        dense_y<R, R, TR>(a.g, (const R*)J.Uin, (R*)J.Uout, J.B, (R)J.lam, lb, (R*)lds,
                          p.s == 1 ? a.spd : nullptr);
}

__device__ __forceinline__ unsigned int dense_tiles(const PArgs& p) {
    return (unsigned int)(ptab(p, L_DX)[p.n] + ptab(p, L_DY)[p.n]);
}

// Takes dense tiles until the queue is empty.  Every thread of the block calls it.
template <typename R, int RB, int TR>
__device__ void drain_tiles(const PArgs& p, unsigned char* lds) {
    __shared__ unsigned int s_tile;
    unsigned int total = dense_tiles(p);
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&p.gs->queue[p.s], 1u);
        __syncthreads();
        unsigned int t = s_tile;
        __syncthreads();  // s_tile is rewritten by the next round
        if (t >= total) break;
        dense_tile<R, RB, TR>(p, t, lds);
    }
}

// Barrier k of the launch.  The first `prev` blocks did the phase before it (block 0 is
// always among them) and arrive; the first `next` blocks have work in the phase after it
// and wait until all `prev` arrivals are in.  Block 0 takes part in every barrier, so a
// completed barrier implies that every earlier one completed too.
__device__ void grid_barrier(const PArgs& p, int k, int prev, int next) {
    unsigned int* cnt = &p.gs->arrived[p.s][k];
    int b = blockIdx.x;
    if (b < prev) {
        __threadfence();  // this block's writes of the phase, visible to every block
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (b >= next) return;  // uniform over the block
    if (threadIdx.x == 0) {
        unsigned long long t0 = wall_clock64();
        while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < (unsigned int)prev) {
            if (__hip_atomic_load(&p.gs->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
            if (wall_clock64() - t0 > p.wait_ticks) {
                __hip_atomic_fetch_or(&p.gs->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
    __threadfence();  // the other blocks' writes of the phase, visible to every wavefront here
}

// Number of leading blocks with work in a phase of `ext` virtual blocks (at least block 0,
// at most the whole grid).
__device__ __forceinline__ int busy(int ext) {
    int g = (int)gridDim.x;
    return ext < 1 ? 1 : (ext > g ? g : ext);
}

__device__ __forceinline__ int wide_ext(const PArgs& p, int kind) { return ptab(p, kind)[p.n]; }
__device__ __forceinline__ int box_ext(const PArgs& p) { return (ptab(p, L_BOX)[p.n] + 3) / 4; }
__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }

// Virtual blocks of T_WIDE threads of launch kind `kind`: f(member args, lb, nb); the loop
// is uniform over the block.
template <class F>
__device__ __forceinline__ void each_wide(const PArgs& p, int kind, F&& f) {
    const int* o = ptab(p, kind);
    int total = o[p.n];
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        int u = find_unit(o, p.n, vb);
        f(p.A[u], vb - o[u], o[u + 1] - o[u]);
    }
}

// Virtual blocks of T_BOX threads (one per wavefront) of the box kinds: f(member args, t).
template <class F>
__device__ __forceinline__ void each_box(const PArgs& p, F&& f) {
    const int* o = ptab(p, L_BOX);
    int total = o[p.n];
    int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int vb = blockIdx.x * 4 + w; vb < total; vb += gridDim.x * 4) {
        int u = find_unit(o, p.n, vb);
        f(p.A[u], (vb - o[u]) * T_BOX + lane);
    }
}


template <typename R, int RB, int TR>
__global__ __launch_bounds__(256) void kb_sweep(PArgs p) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[persist_lds<R, TR>()];
    double* spoly = reinterpret_cast<double*>(lds);
    const int s = p.s;
    const int tid = threadIdx.x;
    int bar = 0;  // barrier index within the launch
    // blocks with work in the current phase: the first phase of sweep 0 poses the polygons,
    // that of sweep 1 is the stage-and-wall phase over the box cells
    int prv = busy(s == 0 ? wide_ext(p, L_POSE) : box_ext(p));
    if (s == 0) {
        for (int lev = 0; lev < 2; lev++)
            each_wide(p, L_POSE, [&](const StepArgs& a, int lb, int) { pose_body(a, lev, lb * T_WIDE + tid); });
        { int nx_ = busy(wide_ext(p, L_V1)); grid_barrier(p, bar++, prv, nx_); prv = nx_; }
        each_wide(p, L_V1, [&](const StepArgs& a, int lb, int nb) { geo_stage_split<0>(a, lb, nb, spoly); });
        { int nx_ = busy(wide_ext(p, L_F1)); grid_barrier(p, bar++, prv, nx_); prv = nx_; }
        each_wide(p, L_F1, [&](const StepArgs& a, int lb, int nb) { geo_stage_split<1>(a, lb, nb, spoly); });
        { int nx_ = busy(imax(wide_ext(p, L_C1), wide_ext(p, L_S1))); grid_barrier(p, bar++, prv, nx_); prv = nx_; }
        // cells, and the apertures of both sweeps (they need the faces of all three levels)
        each_wide(p, L_C1, [&](const StepArgs& a, int lb, int nb) { geo_stage_split<2>(a, lb, nb, spoly); });
        for (int sw = 0; sw < 2; sw++)
            each_wide(p, L_S1, [&](const StepArgs& a, int lb, int nb) { swept_block(a, sw, lb, nb, spoly); });
        { int nx_ = busy(box_ext(p)); grid_barrier(p, bar++, prv, nx_); prv = nx_; }
    }
    each_box(p, [&](const StepArgs& a, int t) { stagewall_body<R>(a, s, t); });
    { int nx_ = busy(box_ext(p)); grid_barrier(p, bar++, prv, nx_); prv = nx_; }
    each_box(p, [&](const StepArgs& a, int t) {
        const SweepJob& J = a.sw[s];
        if (box_empty_dev(J.B)) return;
        if (J.dir == 0) patch<0, R>(a.g, J, stage_of(a, s), a.ncol, t);
        else patch<1, R>(a.g, J, stage_of(a, s), a.ncol, t);
    });
    { int nx_ = busy(box_ext(p)); grid_barrier(p, bar++, prv, nx_); prv = nx_; }
    each_box(p, [&](const StepArgs& a, int t) {
        const SweepJob& J = a.sw[s];
        if (box_empty_dev(J.B)) return;
        double lost[4];
        cover<R>(a.g, J, a.S, t, lost);
    });
    { int nx_ = busy(box_ext(p)); grid_barrier(p, bar++, prv, nx_); prv = nx_; }
    for (int round = 0; round < 2; round++) {
        each_box(p, [&](const StepArgs& a, int t) {
            const SweepJob& J = a.sw[s];
            if (box_empty_dev(J.B)) return;
            double lost[4];
            fix<R>(a.g, J, a.S, round, a.ncol, a.status, t, lost);
        });
        if (round == 0 || s == 1) { int nx_ = busy(box_ext(p)); grid_barrier(p, bar++, prv, nx_); prv = nx_; }
    }
    if (s == 1) each_box(p, [&](const StepArgs& a, int t) { box_speeds<R>(a, s, t); });
    drain_tiles<R, RB, TR>(p, lds);  // the dense tiles not taken yet
    // the last block to finish resets the tile queue and, after the second sweep, gathers
    // the status words (with the barrier error flag) for one read-back
    __shared__ int s_last;
    __syncthreads();
    if (tid == 0) {
        unsigned int old = __hip_atomic_fetch_add(&p.gs->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = old == gridDim.x - 1u;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    if (s == 1) {
        const int* od = ptab(p, L_DX);
        const int* oy = ptab(p, L_DY);
        const int* ob = ptab(p, L_BOX);
        for (int u = 0; u < p.n; u++) {
            const int* o = p.A[u].sw[1].dir == 0 ? od : oy;
            combine_speeds(p.A[u], o[u + 1] - o[u], ob[u + 1] - ob[u], p.gather, u);
        }
        __syncthreads();
        if (__hip_atomic_load(&p.gs->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
            for (int u = tid; u < p.n; u += blockDim.x) p.gather[2 * u] |= 8u;
    }
    if (tid < MAX_BARRIERS) p.gs->arrived[s][tid] = 0u;
    if (tid == 0) {
        p.gs->queue[s] = 0u;
        p.gs->done = 0u;
    }
}

}  // namespace cc
