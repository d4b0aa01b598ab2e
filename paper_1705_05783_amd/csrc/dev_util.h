// Device helpers shared by the libcams kernels: cell coordinates, the six
// faces of a cell in the 7-point stencil, and deterministic reductions.
#pragma once

#include <hip/hip_runtime.h>

#include "cams_internal.h"

namespace cams {

struct Cell {
    int i, j, k;
};

__device__ __forceinline__ Cell cell_of(const GridDev &g, int n)
{
    Cell c;
    c.i = n % g.nx;
    int t = n / g.nx;
    c.j = t % g.ny;
    c.k = t / g.ny;
    return c;
}

// Wave-level sum (lane 0 holds the result), fixed shuffle tree.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Workgroup sum of NT threads (NT multiple of 64); result valid in thread 0.
// Deterministic: fixed tree inside each wave, then waves in index order.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int t = 0; t < NT / 64; ++t) s += sh[t];
    }
    __syncthreads();
    return s;
}

__device__ __forceinline__ int node_index(const GridDev &g, int a, int b, int c)
{
    return a + g.nb[0] * (b + g.nb[1] * c);
}

// Cell of this thread in a flat batched launch, or -1; also returns the
// instance descriptor and skips instances that have converged.
__device__ __forceinline__ int flat_cell(const InstDev *__restrict__ inst, const WorkItem *__restrict__ work,
                                         const InstDev *&d)
{
    const WorkItem w = work[blockIdx.x];
    d = &inst[w.inst];
    if (d->a.ictl[C_DONE]) return -1;
    const int n = w.blk * kBlock + threadIdx.x;
    return n < d->g.N ? n : -1;
}

}  // namespace cams
