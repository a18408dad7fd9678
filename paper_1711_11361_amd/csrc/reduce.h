// State conversion, global time-step reduction and conservation totals.
#pragma once
#include "cc_device.h"

namespace cc {

// U = alpha Q from primitive fields (rho, u, v, p), SoA planes of nx*ny doubles.
template <typename R>
__global__ void k_prim_to_u(Grid g, const double* __restrict__ alpha, const double* __restrict__ prim,
                            R* __restrict__ U) {
    size_t nc = (size_t)g.nx * g.ny;
    size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nc) return;
    double r = prim[k], u = prim[nc + k], v = prim[2 * nc + k], p = prim[3 * nc + k];
    double a = alpha[k];
    double q[4] = {r, r * u, r * v, p / (g.gamma - 1.0) + 0.5 * r * (u * u + v * v)};
#pragma unroll
    for (int m = 0; m < 4; m++) U[m * nc + k] = (R)(a * q[m]);
}

__global__ void k_fill_f64(size_t n, double v, double* __restrict__ p) {
    size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

// Apertures of a level's faces from their solid intervals.
__global__ void k_interval_beta(size_t n, const double2* __restrict__ iv, double* __restrict__ beta) {
    size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) beta[k] = interval_beta(iv[k]);
}

template <typename R>
__global__ void k_copy_u(size_t n, const double* __restrict__ src, R* __restrict__ dst) {
    size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = (R)src[k];
}

template <typename R>
__global__ void k_u_to_f64(size_t n, const R* __restrict__ src, double* __restrict__ dst) {
    size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = (double)src[k];
}

// Primitive fields of the level-n state; solid or emptied cells give zeros.
template <typename R>
__global__ void k_u_to_prim(Grid g, const double* __restrict__ alpha, const R* __restrict__ U,
                            double* __restrict__ prim) {
    size_t nc = (size_t)g.nx * g.ny;
    size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nc) return;
    double a = alpha[k];
    double q[4];
#pragma unroll
    for (int m = 0; m < 4; m++) q[m] = (double)U[m * nc + k];
    if (a > 0.0 && q[0] > 0.0) {
#pragma unroll
        for (int m = 0; m < 4; m++) q[m] = q[m] / a;
        prim[k] = q[0];
        prim[nc + k] = q[1] / q[0];
        prim[2 * nc + k] = q[2] / q[0];
        prim[3 * nc + k] = pressure(q, g.gamma);
    } else {
        prim[k] = prim[nc + k] = prim[2 * nc + k] = prim[3 * nc + k] = 0.0;
    }
}

// Maximum signal speeds max(|u|+a), max(|v|+a) over live cells.  Non-negative doubles
// order like their bit patterns, so the maximum is an exact, order-independent integer
// atomic max; a non-finite or negative-pressure cell produces a NaN pattern above every
// finite speed, which the host reports as a state error.
__device__ __forceinline__ unsigned long long wave_max64(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

constexpr int CFL_BLOCKS = 512;

// Time-step reduction: block lb of nb grid-strides over the cells and writes its maxima of
// |u|+a along x and y over the live cells (alpha > 0 with content) to part[2 lb .. 2 lb + 1]
// as bit patterns (non-negative doubles order like their bit patterns; NaN is mapped above
// infinity, so a non-finite state surfaces in the maximum).
template <typename R>
__device__ void cfl_block(const Grid& g, const double* __restrict__ alpha, const R* __restrict__ U,
                          unsigned long long* __restrict__ part, int lb, int nb) {
    __shared__ unsigned long long sx_[4], sy_[4];
    size_t nc = (size_t)g.nx * g.ny;
    unsigned long long mx = 0ull, my = 0ull;
    for (size_t k = (size_t)lb * blockDim.x + threadIdx.x; k < nc; k += (size_t)nb * blockDim.x) {
        R u[4];
#pragma unroll
        for (int m = 0; m < 4; m++) u[m] = U[m * nc + k];
        unsigned long long bx, by;
        speed_bits(u, alpha[k], g.gamma, bx, by);
        mx = bx > mx ? bx : mx;
        my = by > my ? by : my;
    }
    mx = wave_max64(mx);
    my = wave_max64(my);
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sx_[w] = mx;
        sy_[w] = my;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < (int)(blockDim.x >> 6); q++) {
            mx = sx_[q] > mx ? sx_[q] : mx;
            my = sy_[q] > my ? sy_[q] : my;
        }
        part[2 * lb] = mx;
        part[2 * lb + 1] = my;
    }
}

// Maximum over nparts block partials (one block of 256 threads).
__device__ void cfl_combine(int nparts, const unsigned long long* __restrict__ part,
                            unsigned long long* __restrict__ out) {
    __shared__ unsigned long long sx_[4], sy_[4];
    unsigned long long mx = 0ull, my = 0ull;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) {
        unsigned long long a = part[2 * k], b = part[2 * k + 1];
        mx = a > mx ? a : mx;
        my = b > my ? b : my;
    }
    mx = wave_max64(mx);
    my = wave_max64(my);
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sx_[w] = mx;
        sy_[w] = my;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < (int)(blockDim.x >> 6); q++) {
            mx = sx_[q] > mx ? sx_[q] : mx;
            my = sy_[q] > my ? sy_[q] : my;
        }
        out[0] = mx;
        out[1] = my;
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_cfl(Grid g, const double* __restrict__ alpha, const R* __restrict__ U,
                                             unsigned long long* __restrict__ part) {
    cfl_block<R>(g, alpha, U, part, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_cfl_final(int nparts, const unsigned long long* __restrict__ part,
                                                   unsigned long long* __restrict__ smax) {
    cfl_combine(nparts, part, smax);
}

// dt = cfl min(hx / Sx, hy / Sy) on the device from the reduced speed maxima (bit
// patterns) and the body's largest vertex speeds along x and y (computed by the host for
// the same time), with the host path's operations, so both give the same dt; 0 when the
// state is not finite or the status word holds an error (bits 2 and 8; bit 1 is only a
// report).
__global__ void k_cfl_dt(const unsigned long long* __restrict__ smax, const unsigned int* __restrict__ status,
                         double wsx, double wsy, double hx, double hy, double cfl, double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double sx = __longlong_as_double((long long)smax[0]), sy = __longlong_as_double((long long)smax[1]);
    bool bad = (*status & 14u) != 0u || !isfinite(sx) || !isfinite(sy);
    sx = fmax(sx, wsx);
    sy = fmax(sy, wsy);
    *out = bad ? 0.0 : cfl * fmin(hx / sx, hy / sy);
}

// Deterministic sums: each block reduces a fixed contiguous chunk with a fixed tree; a
// second single-block pass adds the partials in block order.
constexpr int RT = 256;

template <typename R>
__global__ __launch_bounds__(RT) void k_sum_partial(size_t n, int comps, const R* __restrict__ U, size_t chunk,
                                                    double* __restrict__ part) {
    __shared__ double s[RT];
    int c = blockIdx.y;
    size_t b0 = (size_t)blockIdx.x * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
    double acc = 0.0;
    for (size_t k = b0 + threadIdx.x; k < b1; k += RT) acc += (double)U[(size_t)c * n + k];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = RT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)c * gridDim.x + blockIdx.x] = s[0];
    (void)comps;
}

// out[c] = (sum of the partials of component c) * scale
__global__ __launch_bounds__(RT) void k_sum_final(int nblocks, const double* __restrict__ part, double scale,
                                                  double* __restrict__ out) {
    __shared__ double s[RT];
    int c = blockIdx.x;
    double acc = 0.0;
    for (int k = threadIdx.x; k < nblocks; k += RT) acc += part[(size_t)c * nblocks + k];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = RT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = s[0] * scale;
}

}  // namespace cc
