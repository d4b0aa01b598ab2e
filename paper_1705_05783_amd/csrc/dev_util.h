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

// v from the lane that DPP control `ctrl` selects (both 32-bit halves).
template <int ctrl>
__device__ __forceinline__ double dpp_f64(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, ctrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), ctrl, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double read_lane_f64(double v, int lane)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Wave-level sum over all 64 lanes (every lane must be active; every lane
// gets the result), fixed tree: pairs, quads, half rows and rows of 16 by
// DPP exchanges (each partner adds the same two values, so all lanes of a
// row agree), then the four row sums as (r0 + r1) + (r2 + r3).
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);   // row_half_mirror
    v += dpp_f64<0x140>(v);   // row_mirror
    return (read_lane_f64(v, 0) + read_lane_f64(v, 16)) + (read_lane_f64(v, 32) + read_lane_f64(v, 48));
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

// Prolongation (Eq. (12)) at one cell: sum over the 8 coarse nodes that
// bracket cell n = (i, j, k) of P_t[n] xc[node t], skipping zero weights and
// nodes past the last; 0 at Dirichlet cells.  The basis is FP64 (summed in
// FP64) or FP32 / bfloat16 bits (summed in FP32).  Branch-free: the mask,
// node-table and basis loads go out together, then the coarse values.  Every
// prolongation of the solve (standalone or inside the first smoothing step)
// goes through here, so all agree bit for bit.
template <class TP>
struct BasisAcc {
    using T = float;
};
template <>
struct BasisAcc<double> {
    using T = double;
};
__device__ __forceinline__ double basis_load(const double *P, size_t i) { return P[i]; }
__device__ __forceinline__ float basis_load(const float *P, size_t i) { return P[i]; }
__device__ __forceinline__ float basis_load(const uint16_t *P, size_t i)
{
    return __uint_as_float((uint32_t)P[i] << 16);
}

// The loads of one cell's prolongation that do not depend on the coarse
// vector (mask, node tables, basis), and the combination with the coarse
// values (from device memory or a copy in LDS).
template <class TP>
struct ProlongIn {
    typename BasisAcc<TP>::T w[8];
    int a, b, c;
    bool keep;
};

template <class TP>
__device__ __forceinline__ ProlongIn<TP> prolong_load(const GridDev &g, const TP *__restrict__ P,
                                                     const uint8_t *__restrict__ dm, int n, int i, int j, int k)
{
    ProlongIn<TP> in;
    in.keep = !dm[n];
    in.a = g.lo[0][i];
    in.b = g.lo[1][j];
    in.c = g.lo[2][k];
#pragma unroll
    for (int t = 0; t < 8; ++t) in.w[t] = basis_load(P, (size_t)t * g.N + n);
    return in;
}

template <class TP>
__device__ __forceinline__ typename BasisAcc<TP>::T prolong_combine(const GridDev &g, const ProlongIn<TP> &in,
                                                                    const double *xc)
{
    using A = typename BasisAcc<TP>::T;
    double xv[8];
    bool use[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int na = in.a + (t & 1), nb = in.b + ((t >> 1) & 1), nc = in.c + ((t >> 2) & 1);
        const bool inn = na < g.nb[0] && nb < g.nb[1] && nc < g.nb[2];
        xv[t] = xc[inn ? node_index(g, na, nb, nc) : 0];
        use[t] = inn;
    }
    A s = A(0);
#pragma unroll
    for (int t = 0; t < 8; ++t) s = (use[t] && in.w[t] != A(0)) ? s + in.w[t] * (A)xv[t] : s;
    return in.keep ? s : A(0);
}

template <class TP>
__device__ __forceinline__ typename BasisAcc<TP>::T prolong_at(const GridDev &g, const TP *__restrict__ P,
                                                               const uint8_t *__restrict__ dm,
                                                               const double *__restrict__ xc, int n, int i, int j,
                                                               int k)
{
    return prolong_combine(g, prolong_load(g, P, dm, n, i, j, k), xc);
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
    // four independent sums per thread, so that four loads are in flight
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    int t = threadIdx.x;
    for (; t + 3 * kStopThreads < nparts; t += 4 * kStopThreads)
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] += partial[t + u * kStopThreads];
    for (; t < nparts; t += kStopThreads) a[0] += partial[t];
    const double s = block_sum<kStopThreads>((a[0] + a[1]) + (a[2] + a[3]), sh);
    if (threadIdx.x != 0) return;
    const int it = ictl[C_IT];
    if (it == 0) scal[S_R0N2] = s;
    const double r0n2 = it == 0 ? s : scal[S_R0N2];
    scal[S_RN2] = s;
    int outcome = -1;
    if (!(s < 1e300))                          // NaN or Inf
        outcome = 2;
    else if (s <= rtol2 * r0n2 || s <= scal[S_ATOL2] || r0n2 == 0.0)
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
