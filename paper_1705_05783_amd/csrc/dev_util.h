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

// Bijection from the dispatch id to a logical block id such that each of the
// 8 XCDs (which receive dispatch ids round-robin) works on one contiguous
// range of logical blocks, so neighbouring blocks share one L2.
__device__ __forceinline__ int xcd_swizzle(int wg, int n)
{
    const int q = n / 8, rem = n % 8;
    const int xcd = wg % 8, slot = wg / 8;
    return xcd < rem ? xcd * (q + 1) + slot : rem * (q + 1) + (xcd - rem) * q + slot;
}

__device__ __forceinline__ int node_index(const GridDev &g, int a, int b, int c)
{
    return a + g.nb[0] * (b + g.nb[1] * c);
}

// Loop of a persistent batched kernel over its work items: blockIdx.x,
// blockIdx.x + gridDim.x, ... below the device-side count *nwork (uniform
// over the workgroup).
#define CAMS_FOR_ITEMS(t, nwork) for (int t = blockIdx.x, t##_end = *(nwork); t < t##_end; t += gridDim.x)

// Cell of this thread for work item w of a flat batched launch (w.blk =
// block of kBlock cells), or -1 past the instance's cells or once the
// instance has stopped; also returns the instance descriptor.
__device__ __forceinline__ int flat_cell(const InstDev *__restrict__ inst, const WorkItem w, const InstDev *&d)
{
    d = &inst[w.inst];
    if (d->a.ictl[C_DONE]) return -1;
    const int n = w.blk * kBlock + threadIdx.x;
    return n < d->g.N ? n : -1;
}

// ||r||^2 from the residual kernel's nparts partials (in index order, then
// a fixed tree) and the stopping test of the C-AMS iteration, by one
// workgroup of kStopThreads threads: outcome 0 converged (||r||^2 <= rtol2
// ||r0||^2, or r0 = 0), 1 iteration limit, 2 non-finite norm; otherwise the
// iteration counter advances.  Every caller uses the same thread count, so
// the norm is the same bit for bit wherever the test runs.
constexpr int kStopThreads = 256;

__device__ __forceinline__ void stop_test(const double *__restrict__ partial, int nparts, int32_t *ictl,
                                          double *scal, double rtol2, int maxit, double *sh)
{
    double u = 0.0;
    for (int t = threadIdx.x; t < nparts; t += kStopThreads) u += partial[t];
    const double s = block_sum<kStopThreads>(u, sh);
    if (threadIdx.x != 0) return;
    const int it = ictl[C_IT];
    if (it == 0) scal[S_R0N2] = s;
    const double r0n2 = it == 0 ? s : scal[S_R0N2];
    scal[S_RN2] = s;
    int outcome = -1;
    if (!(s < 1e300))                          // NaN or Inf
        outcome = 2;
    else if (s <= rtol2 * r0n2 || r0n2 == 0.0)
        outcome = 0;
    else if (it >= maxit)
        outcome = 1;
    if (outcome < 0) {
        ictl[C_IT] = it + 1;
        return;
    }
    ictl[C_OUTCOME] = outcome;
    ictl[C_DONE] = 1;
}

}  // namespace cams
