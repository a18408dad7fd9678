// Compacted lists of the cells of a box that satisfy a predicate, as linear indices j nx + i
// in increasing order: the cut cells of a level (cells whose four faces are neither all open
// nor all closed) and the wall cells of the surface pressure.  Both lie in the level's
// region box, so only the box is scanned: the box is cut into CUT_BLOCKS contiguous chunks
// of its row-major cell order (which is increasing in j nx + i), each block counts its
// chunk's cells, one block turns the counts into offsets, and each block writes its chunk's
// cells in order.  The result does not depend on timing.
#pragma once
#include "sweep.h"

namespace cc {

constexpr int CUT_T = 256, CUT_BLOCKS = 1024;

// The cut cells of level L.
struct CutCells {
    Grid g;
    Level L;
    __device__ __forceinline__ bool operator()(int i, int j) const { return cell_cut_f(cell_faces(g, L, i, j)); }
};

template <class P>
__device__ __forceinline__ bool box_cell_in(const P& pred, const Box& R, int t, int& lin) {
    int i = R.i0 + t % R.w(), j = R.j0 + t / R.w();
    lin = j * pred.g.nx + i;
    return pred(i, j);
}

// Block b: its chunk of the box's cells, [b chunk, (b + 1) chunk).
template <class P>
__global__ __launch_bounds__(CUT_T) void k_list_count(P pred, Box R, int chunk, int* __restrict__ counts) {
    int cells = R.w() * R.h();
    int t0 = blockIdx.x * chunk, t1 = min(t0 + chunk, cells);
    int n = 0;
    for (int t = t0 + (int)threadIdx.x; t < t1; t += CUT_T) {
        int lin;
        n += box_cell_in(pred, R, t, lin) ? 1 : 0;
    }
    __shared__ int s[CUT_T];
    s[threadIdx.x] = n;
    __syncthreads();
    for (int w = CUT_T / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = s[0];
}

// One block: exclusive offsets of the nb counts (in place) and the total.
__global__ __launch_bounds__(CUT_T) void k_cut_scan(int nb, int* __restrict__ counts, int* __restrict__ total) {
    __shared__ int s[CUT_T];
    int per = (nb + CUT_T - 1) / CUT_T, b0 = threadIdx.x * per, b1 = min(b0 + per, nb);
    int sum = 0;
    for (int b = b0; b < b1; b++) sum += counts[b];
    s[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {  // offsets of the threads' runs
        int acc = 0;
        for (int q = 0; q < CUT_T; q++) {
            int v = s[q];
            s[q] = acc;
            acc += v;
        }
        *total = acc;
    }
    __syncthreads();
    int acc = s[threadIdx.x];
    for (int b = b0; b < b1; b++) {
        int v = counts[b];
        counts[b] = acc;
        acc += v;
    }
}

// Block b writes its chunk's listed cells from offset counts[b] on, in increasing order:
// CUT_T cells at a time, each wavefront's listed lanes counted with a ballot.
template <class P>
__global__ __launch_bounds__(CUT_T) void k_list_write(P pred, Box R, int chunk, const int* __restrict__ counts,
                                                      int* __restrict__ out) {
    __shared__ int wsum[CUT_T / WAVE];
    int cells = R.w() * R.h();
    int t0 = blockIdx.x * chunk, t1 = min(t0 + chunk, cells);
    int base = counts[blockIdx.x];
    int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    for (int s0 = t0; s0 < t1; s0 += CUT_T) {
        int t = s0 + (int)threadIdx.x, lin = 0;
        bool cut = t < t1 && box_cell_in(pred, R, t, lin);
        unsigned long long mask = __ballot(cut);
        if (lane == 0) wsum[wv] = __popcll(mask);
        __syncthreads();
        int before = 0, all = 0;
        for (int q = 0; q < CUT_T / WAVE; q++) {
            before += q < wv ? wsum[q] : 0;
            all += wsum[q];
        }
        if (cut) out[base + before + __popcll(mask & ((1ull << lane) - 1ull))] = lin;
        base += all;
        __syncthreads();  // wsum is rewritten by the next tile
    }
}

}  // namespace cc
