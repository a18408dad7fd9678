// Surface loads: force and moment of the gas on the body at level n, from the cut cells'
// wall pressures (post-processing of the pitching-aerofoil case of Sec. 3.6).  Per cell
// with fluid content and a wall: p* of the wall Riemann problem (Eq. riemann_wallvel with
// HLLC/Davis speeds, reading R9) between the cell state U/alpha and its mirror image moving
// with the body at the cell's wall point, times the level's effective wall normal
// N = ((beta_W - beta_E) h_y, (beta_S - beta_N) h_x) (reading R12; pointing into the body).
// Sums: Fx, Fy, Mz about the body's pose origin, and sum p* |N| (the scale against which
// the rounding of the other three is measured).  Deterministic order: per thread over a
// fixed stride, per block through a fixed tree, per launch over the blocks in order.
#pragma once
#include "sweep.h"

namespace cc {

constexpr int LOADS_T = 256;
constexpr int LOADS_MAX_BLOCKS = 128;

struct BodyVel {
    double vx, vy, thd, cx, cy;  // rigid velocity v + thd z x (X - c) at time t
};

struct LoadsArgs {
    Grid g;
    Level L;    // level n
    Box reg;    // the cells that may differ from fluid
    BodyVel bv[MAX_BODIES];  // each body's velocity (one body: bv[0])
    int body;   // several bodies: the wall cells of this body only, moments about its origin
};

// The body of wall cell k (several bodies: the one the level says cuts it).
__device__ __forceinline__ int loads_body(const LoadsArgs& a, size_t k) {
    if (!a.L.cbody) return 0;
    int b = a.L.cbody[k];
    return b >= 0 ? b : 0;
}

// A wall cell: fluid content and a non-zero effective wall normal (Nx, Ny).
__device__ __forceinline__ bool wall_cell(const Grid& g, const Level& L, double al, double u0, int i, int j,
                                          CellFaces& f, double& Nx, double& Ny) {
    if (!(al > 0.0) || !(u0 > 0.0)) return false;
    f = cell_faces(g, L, i, j);
    Nx = (interval_beta(f.f[0]) - interval_beta(f.f[1])) * g.hy;
    Ny = (interval_beta(f.f[2]) - interval_beta(f.f[3])) * g.hx;
    return !(Nx == 0.0 && Ny == 0.0);
}

// p* of wall cell (i, j) (linear index k) and its wall point (wx, wy).
template <typename R>
__device__ __forceinline__ double wall_pressure(const LoadsArgs& a, const R* __restrict__ U, int i, int j,
                                                size_t k, double al, const CellFaces& f, double Nx, double Ny,
                                                double& wx, double& wy) {
    const Grid& g = a.g;
    size_t nc = (size_t)g.nx * g.ny;
    double q[4];
#pragma unroll
    for (int m = 0; m < 4; m++) q[m] = (double)U[m * nc + k] / al;
    double nn = sqrt(Nx * Nx + Ny * Ny);
    wall_point(g, f, i, j, &wx, &wy);
    const BodyVel& v = a.bv[loads_body(a, k)];
    double uwx = v.vx - v.thd * (wy - v.cy);
    double uwy = v.vy + v.thd * (wx - v.cx);
    double ps, rs;
    wall_riemann(q, Nx / nn, Ny / nn, uwx, uwy, g.gamma, &ps, &rs);
    return ps;
}

template <typename R>
__global__ __launch_bounds__(LOADS_T) void k_loads(LoadsArgs a, const R* __restrict__ U, double* __restrict__ part) {
    const Grid& g = a.g;
    int w = a.reg.w(), h = a.reg.h();
    int cells = w > 0 && h > 0 ? w * h : 0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = blockIdx.x * LOADS_T + threadIdx.x; t < cells; t += gridDim.x * LOADS_T) {
        int i = a.reg.i0 + t % w, j = a.reg.j0 + t / w;
        size_t k = (size_t)j * g.nx + i;
        double al = a.L.alpha[k];
        CellFaces f;
        double Nx, Ny;
        if (!wall_cell(g, a.L, al, (double)U[k], i, j, f, Nx, Ny)) continue;
        if (a.L.cbody && a.L.cbody[k] != a.body) continue;
        double wx, wy;
        double ps = wall_pressure(a, U, i, j, k, al, f, Nx, Ny, wx, wy);
        const BodyVel& o = a.bv[a.body];
        acc[0] += ps * Nx;
        acc[1] += ps * Ny;
        acc[2] += (wx - o.cx) * (ps * Ny) - (wy - o.cy) * (ps * Nx);
        acc[3] += ps * sqrt(Nx * Nx + Ny * Ny);
    }
    __shared__ double sh[4][LOADS_T];
#pragma unroll
    for (int m = 0; m < 4; m++) sh[m][threadIdx.x] = acc[m];
    __syncthreads();
    for (int s = LOADS_T / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int m = 0; m < 4; m++) sh[m][threadIdx.x] += sh[m][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// The blocks' partial sums in block order (one thread per quantity).
__global__ void k_loads_final(int nblocks, const double* __restrict__ part, double* __restrict__ out) {
    if (threadIdx.x >= 4) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; b++) s += part[4 * b + threadIdx.x];
    out[threadIdx.x] = s;
}

// The wall cells of level L for the list kernels (lists.h).
template <typename R>
struct WallCells {
    Grid g;
    Level L;
    const R* U;
    __device__ __forceinline__ bool operator()(int i, int j) const {
        size_t k = (size_t)j * g.nx + i;
        CellFaces f;
        double Nx, Ny;
        return wall_cell(g, L, L.alpha[k], (double)U[k], i, j, f, Nx, Ny);
    }
};

// Record t of the wall pressure distribution: listed cell list[t] (t < min(*n, max)) as
// six values: linear index, wall point x and y, p*, Nx, Ny.
template <typename R>
__global__ __launch_bounds__(LOADS_T) void k_wall_records(LoadsArgs a, const R* __restrict__ U,
                                                          const int* __restrict__ list, const int* __restrict__ n,
                                                          int max, double* __restrict__ out) {
    int t = blockIdx.x * LOADS_T + threadIdx.x;
    int cnt = *n < max ? *n : max;
    if (t >= cnt) return;
    int k = list[t];
    int i = k % a.g.nx, j = k / a.g.nx;
    double al = a.L.alpha[k];
    CellFaces f;
    double Nx = 0.0, Ny = 0.0;
    (void)wall_cell(a.g, a.L, al, (double)U[k], i, j, f, Nx, Ny);
    double wx, wy;
    double ps = wall_pressure(a, U, i, j, (size_t)k, al, f, Nx, Ny, wx, wy);
    double* r = out + 6 * (size_t)t;
    r[0] = (double)k;
    r[1] = wx;
    r[2] = wy;
    r[3] = ps;
    r[4] = Nx;
    r[5] = Ny;
}

}  // namespace cc
