// Iteration control of the C-AMS solve (Table "cams" steps 2 and 5) kept on
// the device: the residual kernel computes r = r0 - A d, its norm, and the
// stopping test; every later kernel of the iteration reads the resulting
// `done` flag and returns at once after convergence.  The host can therefore
// enqueue several iterations ahead and look at the flag only now and then.
//
// Reductions are two-stage and deterministic: workgroups write partials, a
// later launch (one workgroup, or the consumer kernel itself) adds them in
// index order.  Kernel boundaries order the stages; no workgroup uses a
// device-scope fence (on a multi-XCD part that writes back the whole L2).
#include "cams_internal.h"
#include "dev_util.h"

namespace cams {

namespace {

__global__ __launch_bounds__(kBlock) void k_iter_reset(int32_t *__restrict__ ictl, double *__restrict__ dp, int N,
                                                        int nctl)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < N) dp[t] = 0.0;
    if (t < nctl) ictl[t] = 0;
}

// v0 + (v[0] + ... + v[NV-1] once `fold` is set), added in that order; the
// pending corrections are FP64 or, in the mixed-precision solve, FP32.  The
// NV pointers are valid whether or not `fold` is set, so all NV + 1 loads
// are issued together and none waits on a branch.
template <class TA, int NV>
struct Pending {
    const double *v0;
    const TA *v[3];
    bool fold;
    __device__ __forceinline__ double operator()(int m) const
    {
        double s = v0[m];
        TA a[NV > 0 ? NV : 1];
#pragma unroll
        for (int q = 0; q < NV; ++q) a[q] = v[q][m];
#pragma unroll
        for (int q = 0; q < NV; ++q) s = fold ? s + (double)a[q] : s;
        return s;
    }
};

// The non-null pointers of (a0, a1, a2) in order; returns their count.
template <class TA>
int compact_pending(const TA *a0, const TA *a1, const TA *a2, const TA *out[3])
{
    int nv = 0;
    for (const TA *p : {a0, a1, a2})
        if (p) out[nv++] = p;
    for (int q = nv; q < 3; ++q) out[q] = nv ? out[0] : nullptr;
    return nv;
}

// r = r0 - A v at cell n = (i, j, k); writes r (and its FP32 copy rf when
// given) and dp_out = v there, and returns r_n.  A neighbour outside the
// grid is replaced by the cell itself with coupling 0 (s - 0 * v = s), so
// every load is issued at once, without branches.
template <class TA, int NV>
__device__ __forceinline__ double residual_cell(const GridDev &g, const double *__restrict__ W,
                                                const double *__restrict__ diag, const double *__restrict__ r0,
                                                const Pending<TA, NV> &v, double *__restrict__ dp_out,
                                                double *__restrict__ r, float *__restrict__ rf, int n, int i, int j,
                                                int k)
{
    const double *Wx = W, *Wy = W + g.N, *Wz = W + 2 * g.N;
    const bool xm = i > 0, xp = i + 1 < g.nx, ym = j > 0, yp = j + 1 < g.ny, zm = k > 0, zp = k + 1 < g.nz;
    const int nxm = xm ? n - 1 : n, nxp = xp ? n + 1 : n;
    const int nym = ym ? n - g.nx : n, nyp = yp ? n + g.nx : n;
    const int nzm = zm ? n - g.sxy : n, nzp = zp ? n + g.sxy : n;
    const double wxm = Wx[nxm], wxp = Wx[n], wym = Wy[nym], wyp = Wy[n], wzm = Wz[nzm], wzp = Wz[n];
    const double vn = v(n);
    double s = diag[n] * vn;
    s -= (xm ? wxm : 0.0) * v(nxm);
    s -= (xp ? wxp : 0.0) * v(nxp);
    s -= (ym ? wym : 0.0) * v(nym);
    s -= (yp ? wyp : 0.0) * v(nyp);
    s -= (zm ? wzm : 0.0) * v(nzm);
    s -= (zp ? wzp : 0.0) * v(nzp);
    const double rr = r0[n] - s;
    if (r) r[n] = rr;   // null when only the FP32 copy is read afterwards
    if (rf) rf[n] = (float)rr;
    dp_out[n] = vn;
    return rr;
}

// r = r0 - A v over the cells of workgroup `blk` (and its FP32 copy rf when
// given), dp_out = v, and the workgroup's partial of ||r||^2.
template <class TA, int NV>
__device__ __forceinline__ void residual_body(const GridDev &g, const double *__restrict__ W,
                                              const double *__restrict__ diag, const double *__restrict__ r0,
                                              const Pending<TA, NV> &v, double *__restrict__ dp_out,
                                              double *__restrict__ r, float *__restrict__ rf,
                                              double *__restrict__ partial, int blk, double *sh)
{
    const int n = blk * kBlock + threadIdx.x;
    double e2 = 0.0;
    if (n < g.N) {
        const Cell c = cell_of(g, n);
        const double rr = residual_cell(g, W, diag, r0, v, dp_out, r, rf, n, c.i, c.j, c.k);
        e2 = rr * rr;
    }
    const double bs = block_sum<kBlock>(e2, sh);
    if (threadIdx.x == 0) partial[blk] = bs;
}

template <class TA, int NV>
__global__ __launch_bounds__(kBlock) void k_residual_ctl(GridDev g, const double *__restrict__ W,
                                                          const double *__restrict__ diag,
                                                          const double *__restrict__ r0, Pending<TA, NV> v,
                                                          double *__restrict__ dp_out, double *__restrict__ r,
                                                          float *__restrict__ rf, double *__restrict__ partial,
                                                          const int32_t *ictl)
{
    __shared__ double sh[kBlock / 64];
    if (ictl[C_DONE]) return;
    v.fold = ictl[C_IT] > 0;
    // XCD-aware order: the rows above and below a workgroup's rows are read
    // by workgroups of the same XCD, so their lines are found in its L2
    residual_body(g, W, diag, r0, v, dp_out, r, rf, partial, xcd_swizzle(blockIdx.x, gridDim.x), sh);
}

// ||r||^2 from the residual kernel's partials and the stopping test.
constexpr int kFinal = kStopThreads;

__global__ __launch_bounds__(kFinal) void k_finalize_ctl(const double *__restrict__ partial, int nparts,
                                                          int32_t *ictl, double *scal, double rtol2, int maxit)
{
    __shared__ double sh[kFinal / 64];
    if (ictl[C_DONE]) return;
    stop_test(partial, nparts, ictl, scal, rtol2, maxit, sh);
}

// Restriction R r (Eqs. (7), (13), (15)) in two deterministic stages.
// Stage 1, one workgroup per owner box k = (a, b, c): MSFE: the box holds
// the cells whose lower bracketing coarse node is k, so all of them share
// the same 8 bracketing nodes; the workgroup sums P_s[n] r[n] over its
// non-Dirichlet cells for the 8 slots s (slot s = the node k + (s&1,
// (s>>1)&1, s>>2)).  MSFV: the box is the primal block of node k, summed
// with weight 1 into slot 0.  Every cell is read once.
// Stage 2 (node_sum, in the coarse solve): (R r)_k adds, in a fixed order,
// the slot partials that the (up to) 8 boxes around node k hold for it.
// TP: storage type of the basis (double, float, or bfloat16 bits).
template <class TP>
__device__ __forceinline__ double basis_value(const TP *P, size_t i);
template <>
__device__ __forceinline__ double basis_value<double>(const double *P, size_t i) { return P[i]; }
template <>
__device__ __forceinline__ double basis_value<float>(const float *P, size_t i) { return (double)P[i]; }
template <>
__device__ __forceinline__ double basis_value<uint16_t>(const uint16_t *P, size_t i)
{
    return (double)__uint_as_float((uint32_t)P[i] << 16);
}

// One workgroup sums owner box k: cells in x-fastest order, thread-strided;
// per slot a fixed shuffle tree in each wave, then the waves in order.
template <class TP>
__device__ __forceinline__ void restrict_box(const GridDev &g, const uint8_t *__restrict__ dm,
                                             const TP *__restrict__ P, int fe, const double *__restrict__ r,
                                             double *__restrict__ slots, int k, double *sh)
{
    const int ka = k % g.nb[0], kb = (k / g.nb[0]) % g.nb[1], kc = k / (g.nb[0] * g.nb[1]);
    // MSFE: the owner box from the tables; MSFV: the primal block [a r, min((a+1) r, n)) of
    // node k, also when the context was set up for MSFE (the conservative sweep)
    const int x0 = fe ? g.ob[0][ka] : ka * g.r[0], y0 = fe ? g.ob[1][kb] : kb * g.r[1];
    const int z0 = fe ? g.ob[2][kc] : kc * g.r[2];
    const int ex = (fe ? g.ob[0][ka + 1] : min(x0 + g.r[0], g.nx)) - x0;
    const int ey = (fe ? g.ob[1][kb + 1] : min(y0 + g.r[1], g.ny)) - y0;
    const int ez = (fe ? g.ob[2][kc + 1] : min(z0 + g.r[2], g.nz)) - z0;
    const int m = ex * ey * ez;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < m; t += kBlock) {
        const int x = x0 + t % ex, y = y0 + (t / ex) % ey, z = z0 + t / (ex * ey);
        const int n = x + g.nx * (y + g.ny * z);
        const double rn = r[n];
        if (fe) {
            // the basis loads do not wait for the mask: masked cells add 0
            const double wn = dm[n] ? 0.0 : rn;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] += basis_value(P, (size_t)q * g.N + n) * wn;
        } else {
            acc[0] += rn;
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const double v = wave_sum(acc[q]);
        if (lane == 0) sh[q * (kBlock / 64) + w] = v;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double s = 0.0;
        for (int u = 0; u < kBlock / 64; ++u) s += sh[threadIdx.x * (kBlock / 64) + u];
        slots[(size_t)k * 8 + threadIdx.x] = s;
    }
    __syncthreads();   // sh is reused by the caller's next box
}

template <class TP>
__global__ __launch_bounds__(kBlock) void k_restrict(GridDev g, const uint8_t *__restrict__ dm,
                                                      const TP *__restrict__ P, int fe, const double *__restrict__ r,
                                                      double *__restrict__ slots, const int32_t *ictl)
{
    __shared__ double sh[8 * (kBlock / 64)];
    if (ictl[C_DONE]) return;
    restrict_box<TP>(g, dm, P, fe, r, slots, blockIdx.x, sh);
}

// Residual and restriction in one pass, for iterations without
// pre-smoothing (the restriction then acts on the new residual itself): one
// workgroup per owner box k computes, over the box's cells in the order of
// restrict_box, r = r0 - A v as residual_body does, the box's partial of
// ||r||^2 (partial[k]) and its 8 restriction slots from the values just
// computed, so r is not read back and the restriction needs no launch of its
// own.  The slots equal restrict_box's (a masked cell adds P * 0 = +-0).
template <class TA, int NV, class TP, int NT>
__device__ __forceinline__ void residual_restrict_box(const GridDev &g, const double *__restrict__ W,
                                                      const double *__restrict__ diag,
                                                      const double *__restrict__ r0, const Pending<TA, NV> &v,
                                                      double *__restrict__ dp_out, double *__restrict__ r,
                                                      float *__restrict__ rf, double *__restrict__ partial,
                                                      const uint8_t *__restrict__ dm, const TP *__restrict__ P,
                                                      int fe, double *__restrict__ slots, int k, double *sh)
{
    const int ka = k % g.nb[0], kb = (k / g.nb[0]) % g.nb[1], kc = k / (g.nb[0] * g.nb[1]);
    // MSFE: the owner box from the tables; MSFV: the primal block [a r, min((a+1) r, n)) of
    // node k, also when the context was set up for MSFE (the conservative sweep)
    const int x0 = fe ? g.ob[0][ka] : ka * g.r[0], y0 = fe ? g.ob[1][kb] : kb * g.r[1];
    const int z0 = fe ? g.ob[2][kc] : kc * g.r[2];
    const int ex = (fe ? g.ob[0][ka + 1] : min(x0 + g.r[0], g.nx)) - x0;
    const int ey = (fe ? g.ob[1][kb + 1] : min(y0 + g.r[1], g.ny)) - y0;
    const int ez = (fe ? g.ob[2][kc + 1] : min(z0 + g.r[2], g.nz)) - z0;
    const int m = ex * ey * ez;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double e2 = 0.0;
    for (int t = threadIdx.x; t < m; t += NT) {
        const int x = x0 + t % ex, y = y0 + (t / ex) % ey, z = z0 + t / (ex * ey);
        const int n = x + g.nx * (y + g.ny * z);
        // issued with the residual's loads, outside any branch, so that no
        // load waits for another (MSFV reads the basis without using it)
        TP pv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) pv[q] = P[(size_t)q * g.N + n];
        const bool keep = !dm[n];
        const double rn = residual_cell(g, W, diag, r0, v, dp_out, r, rf, n, x, y, z);
        e2 += rn * rn;
        if (fe) {
            const double wn = keep ? rn : 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] += basis_value(pv + q, 0) * wn;
        } else {
            acc[0] += rn;
        }
    }
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const double u = wave_sum(acc[q]);
        if (lane == 0) sh[q * NW + w] = u;
    }
    {
        const double u = wave_sum(e2);
        if (lane == 0) sh[8 * NW + w] = u;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        double s = 0.0;
        for (int u = 0; u < NW; ++u) s += sh[threadIdx.x * NW + u];
        if (threadIdx.x < 8)
            slots[(size_t)k * 8 + threadIdx.x] = s;
        else
            partial[k] = s;
    }
    __syncthreads();   // sh is reused by the caller's next box
}

// Threads per box of the single-problem form: one cell per thread in full
// 8x8x8 boxes.
constexpr int kBoxThreads = 512;

template <class TA, int NV, class TP>
__global__ __launch_bounds__(kBoxThreads) void k_residual_restrict(GridDev g, const double *__restrict__ W,
                                                               const double *__restrict__ diag,
                                                               const double *__restrict__ r0, Pending<TA, NV> v,
                                                               double *__restrict__ dp_out, double *__restrict__ r,
                                                               float *__restrict__ rf, double *__restrict__ partial,
                                                               const uint8_t *__restrict__ dm,
                                                               const TP *__restrict__ P, int fe,
                                                               double *__restrict__ slots, const int32_t *ictl)
{
    __shared__ double sh[9 * (kBoxThreads / 64)];
    if (ictl[C_DONE]) return;
    v.fold = ictl[C_IT] > 0;
    residual_restrict_box<TA, NV, TP, kBoxThreads>(g, W, diag, r0, v, dp_out, r, rf, partial, dm, P, fe, slots,
                                               xcd_swizzle(blockIdx.x, gridDim.x), sh);
}

// The same for a group of consecutive boxes along x (the table gx), so that
// the loads and stores of a wave run along rows of up to 32 cells instead of
// one box's rows of about 8: thread t takes column t % 32 of the group's
// rows and every 16th row (y fastest, then z), so all its cells lie in one
// box.  The per-box sums go through LDS: each wave then reduces some of the
// (box, slot) pairs over that box's threads in a fixed order.  (With
// coarsening ratios up to 8 a box is at most 12 cells wide, so every grid
// has such groups; cams_create checks it.)
constexpr int kRowThreads = 512;

template <class TA, int NV, class TP>
__global__ __launch_bounds__(kRowThreads) void k_residual_restrict_row(
    GridDev g, const double *__restrict__ W, const double *__restrict__ diag, const double *__restrict__ r0,
    Pending<TA, NV> v, double *__restrict__ dp_out, double *__restrict__ r, float *__restrict__ rf,
    double *__restrict__ partial, const uint8_t *__restrict__ dm, const TP *__restrict__ P, int fe,
    double *__restrict__ slots, const int32_t *ictl)
{
    constexpr int NT = kRowThreads, RW = NT / kRowCells;   // rows per pass (16)
    __shared__ double red[9][NT];
    if (ictl[C_DONE]) return;
    v.fold = ictl[C_IT] > 0;
    const int vi = fe ? 1 : 0, ngx = g.ngx[vi];
    const int wg = xcd_swizzle(blockIdx.x, gridDim.x);
    const int gi = wg % ngx, kb = (wg / ngx) % g.nb[1], kc = wg / (ngx * g.nb[1]);
    const int ka0 = g.gx[vi][gi], nbox = g.gx[vi][gi + 1] - ka0;
    auto xs = [&](int b) { return fe ? g.ob[0][b] : min(b * g.r[0], g.nx); };
    const int x0 = xs(ka0), ex = xs(ka0 + nbox) - x0;
    const int y0 = fe ? g.ob[1][kb] : kb * g.r[1], z0 = fe ? g.ob[2][kc] : kc * g.r[2];
    const int ey = (fe ? g.ob[1][kb + 1] : min(y0 + g.r[1], g.ny)) - y0;
    const int ez = (fe ? g.ob[2][kc + 1] : min(z0 + g.r[2], g.nz)) - z0;
    const int tid = threadIdx.x, lx = tid % kRowCells, row0 = tid / kRowCells;
    const bool colx = lx < ex;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double e2 = 0.0;
    const int rows = ey * ez;
    for (int R = row0; colx && R < rows; R += RW) {
        const int x = x0 + lx, y = y0 + R % ey, z = z0 + R / ey;
        const int n = x + g.nx * (y + g.ny * z);
        TP pv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) pv[q] = P[(size_t)q * g.N + n];
        const bool keep = !dm[n];
        const double rn = residual_cell(g, W, diag, r0, v, dp_out, r, rf, n, x, y, z);
        e2 += rn * rn;
        if (fe) {
            const double wn = keep ? rn : 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] += basis_value(pv + q, 0) * wn;
        } else {
            acc[0] += rn;
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) red[q][tid] = acc[q];
    red[8][tid] = e2;
    __syncthreads();
    const int lane = tid & 63, w = tid >> 6;
    for (int pr = w; pr < 9 * nbox; pr += NT / 64) {
        const int b = pr / 9, q = pr % 9;
        const int c0 = xs(ka0 + b) - x0, wdt = xs(ka0 + b + 1) - x0 - c0;
        double sum = 0.0;
        for (int u = lane; u < wdt * RW; u += 64) sum += red[q][(u / wdt) * kRowCells + c0 + u % wdt];
        sum = wave_sum(sum);
        if (lane == 0) {
            const int k = (ka0 + b) + g.nb[0] * (kb + g.nb[1] * kc);
            if (q < 8) slots[(size_t)k * 8 + q] = sum;
            else partial[k] = sum;
        }
    }
}

// Pair form of the row kernel, for grids whose x-extent and box edges along x
// are all even: thread t takes the two cells 2 (t % 16) and 2 (t % 16) + 1
// of a 32-cell row segment, rows t / 16 + 16 i.  Each stencil point of both
// cells is one 16-byte load (two FP64 values; 8 bytes for FP32, 4 for
// BF16, 2 for the mask) instead of two, and only the x-neighbours outside
// the pair take a load of their own, so a cell costs about half the vector
// memory instructions of the row kernel, whose 64-lane loads keep the
// texture address units busy for most of its time.  Both cells lie in one
// box, so a thread keeps one set of box sums.  The residual of each cell is
// formed in the same order as residual_cell, so r is the same bit for bit;
// the box sums add the two cells of a thread first.
constexpr int kPairThreads = 256;
constexpr int kRowPairs = kRowCells / 2;

template <class T>
struct Two {
    T a, b;
};
template <class T>
__device__ __forceinline__ Two<T> load2(const T *__restrict__ p, int n)   // n even
{
    if constexpr (sizeof(T) == 8) {
        const double2 v = *reinterpret_cast<const double2 *>(p + n);
        return {v.x, v.y};
    } else if constexpr (sizeof(T) == 4) {
        const float2 v = *reinterpret_cast<const float2 *>(p + n);
        return {v.x, v.y};
    } else if constexpr (sizeof(T) == 2) {
        const uint32_t v = *reinterpret_cast<const uint32_t *>(p + n);
        return {(T)(v & 0xffffu), (T)(v >> 16)};
    } else {
        const uint16_t v = *reinterpret_cast<const uint16_t *>(p + n);
        return {(T)(v & 0xffu), (T)(v >> 8)};
    }
}

// Pending value at the even cell m and at m + 1, each summed as Pending does.
template <class TA, int NV>
__device__ __forceinline__ Two<double> pending2(const Pending<TA, NV> &v, int m)
{
    const Two<double> b = load2(v.v0, m);
    Two<TA> a[NV > 0 ? NV : 1];
#pragma unroll
    for (int q = 0; q < NV; ++q) a[q] = load2(v.v[q], m);
    double s0 = b.a, s1 = b.b;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        s0 = v.fold ? s0 + (double)a[q].a : s0;
        s1 = v.fold ? s1 + (double)a[q].b : s1;
    }
    return {s0, s1};
}

template <class TA, int NV, class TP>
__global__ __launch_bounds__(kPairThreads) void k_residual_restrict_pair(
    GridDev g, const double *__restrict__ W, const double *__restrict__ diag, const double *__restrict__ r0,
    Pending<TA, NV> v, double *__restrict__ dp_out, double *__restrict__ r, float *__restrict__ rf,
    double *__restrict__ partial, const uint8_t *__restrict__ dm, const TP *__restrict__ P, int fe,
    double *__restrict__ slots, const int32_t *ictl)
{
    constexpr int NT = kPairThreads, RW = NT / kRowPairs;   // rows per pass (16)
    __shared__ double red[9][NT];
    if (ictl[C_DONE]) return;
    v.fold = ictl[C_IT] > 0;
    const int vi = fe ? 1 : 0, ngx = g.ngx[vi];
    const int wg = xcd_swizzle(blockIdx.x, gridDim.x);
    const int gi = wg % ngx, kb = (wg / ngx) % g.nb[1], kc = wg / (ngx * g.nb[1]);
    const int ka0 = g.gx[vi][gi], nbox = g.gx[vi][gi + 1] - ka0;
    auto xs = [&](int b) { return fe ? g.ob[0][b] : min(b * g.r[0], g.nx); };
    const int x0 = xs(ka0), ex = xs(ka0 + nbox) - x0;
    const int y0 = fe ? g.ob[1][kb] : kb * g.r[1], z0 = fe ? g.ob[2][kc] : kc * g.r[2];
    const int ey = (fe ? g.ob[1][kb + 1] : min(y0 + g.r[1], g.ny)) - y0;
    const int ez = (fe ? g.ob[2][kc + 1] : min(z0 + g.r[2], g.nz)) - z0;
    const int tid = threadIdx.x, px = tid % kRowPairs, row0 = tid / kRowPairs;
    const bool colx = 2 * px < ex;
    const double *Wx = W, *Wy = W + g.N, *Wz = W + 2 * g.N;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double e2 = 0.0;
    const int rows = ey * ez;
    for (int R = row0; colx && R < rows; R += RW) {
        const int x = x0 + 2 * px, y = y0 + R % ey, z = z0 + R / ey;
        const int n = x + g.nx * (y + g.ny * z);   // even
        Two<TP> pv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) pv[q] = load2(P + (size_t)q * g.N, n);
        const Two<uint8_t> mk = load2(dm, n);
        // the cells x and x + 1: x + 1 < nx always, x - 1 and x + 2 may be outside
        const bool xm = x > 0, xp = x + 2 < g.nx, ym = y > 0, yp = y + 1 < g.ny, zm = z > 0, zp = z + 1 < g.nz;
        const int nxm = xm ? n - 1 : n, nxp = xp ? n + 2 : n;
        const int nym = ym ? n - g.nx : n, nyp = yp ? n + g.nx : n;
        const int nzm = zm ? n - g.sxy : n, nzp = zp ? n + g.sxy : n;
        const Two<double> wx = load2(Wx, n), wy = load2(Wy, n), wz = load2(Wz, n);
        const Two<double> wym = load2(Wy, nym), wzm = load2(Wz, nzm);
        const double wxm = Wx[nxm];
        const Two<double> dg = load2(diag, n), rz = load2(r0, n);
        const Two<double> vc = pending2(v, n), vym = pending2(v, nym), vyp = pending2(v, nyp);
        const Two<double> vzm = pending2(v, nzm), vzp = pending2(v, nzp);
        const double vxm = v(nxm), vxp = v(nxp);
        // cell x: its +x neighbour is x + 1; cell x + 1: its -x neighbour is x
        double s0 = dg.a * vc.a;
        s0 -= (xm ? wxm : 0.0) * vxm;
        s0 -= wx.a * vc.b;
        s0 -= (ym ? wym.a : 0.0) * vym.a;
        s0 -= (yp ? wy.a : 0.0) * vyp.a;
        s0 -= (zm ? wzm.a : 0.0) * vzm.a;
        s0 -= (zp ? wz.a : 0.0) * vzp.a;
        double s1 = dg.b * vc.b;
        s1 -= wx.a * vc.a;
        s1 -= (xp ? wx.b : 0.0) * vxp;
        s1 -= (ym ? wym.b : 0.0) * vym.b;
        s1 -= (yp ? wy.b : 0.0) * vyp.b;
        s1 -= (zm ? wzm.b : 0.0) * vzm.b;
        s1 -= (zp ? wz.b : 0.0) * vzp.b;
        const double ra = rz.a - s0, rb = rz.b - s1;
        if (r) *reinterpret_cast<double2 *>(r + n) = double2{ra, rb};
        if (rf) *reinterpret_cast<float2 *>(rf + n) = float2{(float)ra, (float)rb};
        *reinterpret_cast<double2 *>(dp_out + n) = double2{vc.a, vc.b};
        e2 += ra * ra;
        e2 += rb * rb;
        if (fe) {
            const double wa = mk.a ? 0.0 : ra, wb = mk.b ? 0.0 : rb;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                acc[q] += basis_value(&pv[q].a, 0) * wa;
                acc[q] += basis_value(&pv[q].b, 0) * wb;
            }
        } else {
            acc[0] += ra;
            acc[0] += rb;
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) red[q][tid] = acc[q];
    red[8][tid] = e2;
    __syncthreads();
    const int lane = tid & 63, w = tid >> 6;
    for (int pr = w; pr < 9 * nbox; pr += NT / 64) {
        const int b = pr / 9, q = pr % 9;
        const int c0 = (xs(ka0 + b) - x0) / 2, wdt = (xs(ka0 + b + 1) - x0) / 2 - c0;
        double sum = 0.0;
        for (int u = lane; u < wdt * RW; u += 64) sum += red[q][(u / wdt) * kRowPairs + c0 + u % wdt];
        sum = wave_sum(sum);
        if (lane == 0) {
            const int k = (ka0 + b) + g.nb[0] * (kb + g.nb[1] * kc);
            if (q < 8) slots[(size_t)k * 8 + q] = sum;
            else partial[k] = sum;
        }
    }
}

// ---- batched forms: one launch covers every instance of a batch; the work
// item of a workgroup names the instance and the block within it, and
// workgroups of instances that have converged return at once.

// Corrections of the previous iteration: d0 (pre-smoothing; NV = 2), then
// d2, which the post-smoothing started from d1 and so holds d1 + d2, or d1
// alone without post-smoothing.  The batch shares n_pre and n_post.
template <class TA, int NV>
__device__ __forceinline__ Pending<TA, NV> pending_of(const InstDev &d, int par, bool fold)
{
    const TA *d0, *d1, *d2;
    if constexpr (sizeof(TA) == 4) {
        d0 = d.a.d0f; d1 = d.a.d1f; d2 = d.a.d2f;
    } else {
        d0 = d.a.d0; d1 = d.a.d1; d2 = d.a.d2;
    }
    const TA *post = d.n_post > 0 ? d2 : d1;
    if constexpr (NV == 2)
        return Pending<TA, NV>{d.a.dp[par], {d0, post, post}, fold};
    else
        return Pending<TA, NV>{d.a.dp[par], {post, post, post}, fold};
}

// NV = 2 with pre-smoothing (d0 and the post correction), else 1.
template <class TA, int NV>
__global__ __launch_bounds__(kBlock) void kb_residual(const InstDev *__restrict__ inst,
                                                       const WorkItem *__restrict__ work, const int32_t *nwork, int par)
{
    __shared__ double sh[kBlock / 64];
    CAMS_FOR_ITEMS(t, nwork)
    {
        const WorkItem w = work[t];
        const InstDev &d = inst[w.inst];
        if (d.a.ictl[C_DONE]) continue;
        const Pending<TA, NV> v = pending_of<TA, NV>(d, par, d.a.ictl[C_IT] > 0);
        float *rf = sizeof(TA) == 4 ? d.a.r1f : nullptr;
        residual_body(d.g, d.a.W, d.a.diag, d.a.r0, v, d.a.dp[par ^ 1], d.a.r, rf, d.a.partial, w.blk, sh);
    }
}

// One workgroup per instance.
__global__ __launch_bounds__(kFinal) void kb_finalize(const InstDev *__restrict__ inst)
{
    __shared__ double sh[kFinal / 64];
    const InstDev &d = inst[blockIdx.x];
    if (d.a.ictl[C_DONE]) return;
    stop_test(d.a.partial, d.nparts, d.a.ictl, d.a.scal, d.rtol2, d.maxit, sh);
}

// Work item = (instance, owner box).
template <class TP>
__global__ __launch_bounds__(kBlock) void kb_restrict(const InstDev *__restrict__ inst,
                                                       const WorkItem *__restrict__ work, const int32_t *nwork)
{
    __shared__ double sh[8 * (kBlock / 64)];
    CAMS_FOR_ITEMS(t, nwork)
    {
        const WorkItem w = work[t];
        const InstDev &d = inst[w.inst];
        if (d.a.ictl[C_DONE]) continue;
        const TP *P;
        if constexpr (sizeof(TP) == 8)
            P = d.a.P;
        else if constexpr (sizeof(TP) == 4)
            P = d.a.P32;
        else
            P = d.a.Pbf;
        restrict_box<TP>(d.g, d.a.dmask, P, d.fe, d.a.r, d.a.slots, w.blk, sh);
    }
}

// Iteration state of every instance back to its start (dp = 0, counters 0);
// work item = (instance, block of kBlock cells).
__global__ __launch_bounds__(kBlock) void kb_reset(const InstDev *__restrict__ inst, const WorkItem *__restrict__ work,
                                                    const int32_t *nwork)
{
    CAMS_FOR_ITEMS(t, nwork)
    {
        const WorkItem w = work[t];
        const InstDev &d = inst[w.inst];
        const int n = w.blk * kBlock + threadIdx.x;
        if (n < d.g.N) d.a.dp[0][n] = 0.0;
        if (w.blk == 0)
            for (int q = threadIdx.x; q < C_NODE + d.g.Nc; q += kBlock) d.a.ictl[q] = 0;
    }
}

// Iteration counters, outcomes and norms of every instance, for one copy to the host.
__global__ __launch_bounds__(kBlock) void kb_gather(const InstDev *__restrict__ inst, int count,
                                                     BatchResult *__restrict__ out)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= count) return;
    const InstDev &d = inst[t];
    BatchResult r;
    r.it = d.a.ictl[C_IT];
    r.done = d.a.ictl[C_DONE];
    r.outcome = d.a.ictl[C_OUTCOME];
    r.status = d.a.status[0];
    r.eps2 = d.a.scal[S_EPS2];
    r.r0n2 = d.a.scal[S_R0N2];
    r.rn2 = d.a.scal[S_RN2];
    out[t] = r;
}

}  // namespace

void launch_iter_reset(cams_ctx *c)
{
    const int nctl = C_NODE + c->g.Nc;
    const int n = c->g.N > nctl ? c->g.N : nctl;
    k_iter_reset<<<(n + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(c->a.ictl, c->a.dp[0], c->g.N, nctl);
}

template <class TA, int NV>
void residual_flat(cams_ctx *c, const double *dp_in, const TA *const pv[3], double *dp_out, float *rf)
{
    const Pending<TA, NV> v{dp_in, {pv[0], pv[1], pv[2]}, false};
    k_residual_ctl<TA, NV><<<(c->g.N + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(
        c->g, c->a.W, c->a.diag, c->a.r0, v, dp_out, c->a.r, rf, c->a.partial, c->a.ictl);
}

template <class TA>
void residual_flat(cams_ctx *c, const double *dp_in, const TA *a0, const TA *a1, const TA *a2, double *dp_out,
                   float *rf)
{
    const TA *pv[3];
    switch (compact_pending(a0, a1, a2, pv)) {
    case 1: residual_flat<TA, 1>(c, dp_in, pv, dp_out, rf); break;
    case 2: residual_flat<TA, 2>(c, dp_in, pv, dp_out, rf); break;
    case 3: residual_flat<TA, 3>(c, dp_in, pv, dp_out, rf); break;
    default: throw HipError(hipErrorInvalidValue, "pending corrections", __LINE__);   // none: not a C-AMS iteration
    }
}

void launch_residual_ctl(cams_ctx *c, const double *dp_in, const double *a0, const double *a1, const double *a2,
                         double *dp_out)
{
    residual_flat<double>(c, dp_in, a0, a1, a2, dp_out, nullptr);
}

void launch_residual_ctl32(cams_ctx *c, const double *dp_in, const float *a0, const float *a1, const float *a2,
                           double *dp_out, float *rf)
{
    residual_flat<float>(c, dp_in, a0, a1, a2, dp_out, rf);
}

template <class TA, int NV>
void residual_restrict(cams_ctx *c, const Pending<TA, NV> &v, double *dp_out, float *rf)
{
    const GridDev &g = c->g;
    const Arrays &a = c->a;
    const int fe = c->opt.restriction == CAMS_R_FE;
    const int ngx = g.ngx[fe];
    // in mixed precision the smoother reads the FP32 copy rf and the
    // restriction uses r in registers, so the FP64 r is not stored
    double *const rout = rf ? nullptr : a.r;
    // groups of boxes per workgroup where they fill at least one round of
    // resident workgroups (FP32 / BF16 at 128^3: 90 -> 77 us per launch;
    // 256x256x128: 358 -> 268 us), else one workgroup per box (64x64x32:
    // 96 groups, 18.8 against 9.5 us)
    const unsigned wgs = (unsigned)ngx * g.nb[1] * g.nb[2];
    if (c->row_pairs[fe] &&
        (int)wgs >= resident_workgroups((const void *)k_residual_restrict_pair<TA, NV, float>, kPairThreads)) {
        if (c->opt.precision == CAMS_MIXED_BF16)
            k_residual_restrict_pair<TA, NV, uint16_t><<<wgs, kPairThreads, 0, c->stream>>>(
                g, a.W, a.diag, a.r0, v, dp_out, rout, rf, a.partial, a.dmask, a.Pbf, fe, a.slots, a.ictl);
        else if (c->opt.precision == CAMS_MIXED_FP32)
            k_residual_restrict_pair<TA, NV, float><<<wgs, kPairThreads, 0, c->stream>>>(
                g, a.W, a.diag, a.r0, v, dp_out, rout, rf, a.partial, a.dmask, a.P32, fe, a.slots, a.ictl);
        else
            k_residual_restrict_pair<TA, NV, double><<<wgs, kPairThreads, 0, c->stream>>>(
                g, a.W, a.diag, a.r0, v, dp_out, rout, rf, a.partial, a.dmask, a.P, fe, a.slots, a.ictl);
        return;
    }
    if ((int)wgs >= resident_workgroups((const void *)k_residual_restrict_row<TA, NV, float>, kRowThreads)) {
        if (c->opt.precision == CAMS_MIXED_BF16)
            k_residual_restrict_row<TA, NV, uint16_t><<<wgs, kRowThreads, 0, c->stream>>>(
                g, a.W, a.diag, a.r0, v, dp_out, rout, rf, a.partial, a.dmask, a.Pbf, fe, a.slots, a.ictl);
        else if (c->opt.precision == CAMS_MIXED_FP32)
            k_residual_restrict_row<TA, NV, float><<<wgs, kRowThreads, 0, c->stream>>>(
                g, a.W, a.diag, a.r0, v, dp_out, rout, rf, a.partial, a.dmask, a.P32, fe, a.slots, a.ictl);
        else
            k_residual_restrict_row<TA, NV, double><<<wgs, kRowThreads, 0, c->stream>>>(
                g, a.W, a.diag, a.r0, v, dp_out, rout, rf, a.partial, a.dmask, a.P, fe, a.slots, a.ictl);
        return;
    }
    if (c->opt.precision == CAMS_MIXED_BF16)
        k_residual_restrict<TA, NV, uint16_t><<<g.Nc, kBoxThreads, 0, c->stream>>>(
            g, a.W, a.diag, a.r0, v, dp_out, rout, rf, a.partial, a.dmask, a.Pbf, fe, a.slots, a.ictl);
    else if (c->opt.precision == CAMS_MIXED_FP32)
        k_residual_restrict<TA, NV, float><<<g.Nc, kBoxThreads, 0, c->stream>>>(
            g, a.W, a.diag, a.r0, v, dp_out, rout, rf, a.partial, a.dmask, a.P32, fe, a.slots, a.ictl);
    else
        k_residual_restrict<TA, NV, double><<<g.Nc, kBoxThreads, 0, c->stream>>>(
            g, a.W, a.diag, a.r0, v, dp_out, rout, rf, a.partial, a.dmask, a.P, fe, a.slots, a.ictl);
}

// Without pre-smoothing at most two corrections are pending (d1 and d2 of
// the red-black smoother's post-smoothing).
template <class TA>
void residual_restrict(cams_ctx *c, const double *dp_in, const TA *a0, const TA *a1, const TA *a2, double *dp_out,
                       float *rf)
{
    const TA *pv[3];
    switch (compact_pending(a0, a1, a2, pv)) {
    case 1: residual_restrict<TA, 1>(c, Pending<TA, 1>{dp_in, {pv[0], pv[1], pv[2]}, false}, dp_out, rf); break;
    case 2: residual_restrict<TA, 2>(c, Pending<TA, 2>{dp_in, {pv[0], pv[1], pv[2]}, false}, dp_out, rf); break;
    default: throw HipError(hipErrorInvalidValue, "pending corrections", __LINE__);
    }
}

void launch_residual_restrict(cams_ctx *c, const double *dp_in, const double *a0, const double *a1,
                              const double *a2, double *dp_out)
{
    residual_restrict<double>(c, dp_in, a0, a1, a2, dp_out, nullptr);
}

void launch_residual_restrict32(cams_ctx *c, const double *dp_in, const float *a0, const float *a1, const float *a2,
                                double *dp_out, float *rf)
{
    residual_restrict<float>(c, dp_in, a0, a1, a2, dp_out, rf);
}

void launch_finalize_ctl(cams_ctx *c, int nparts)
{
    const double rt = c->opt.lin_rtol;
    k_finalize_ctl<<<1, kFinal, 0, c->stream>>>(c->a.partial, nparts, c->a.ictl, c->a.scal, rt * rt,
                                                c->opt.lin_maxit);
}

void launch_restrict(cams_ctx *c, const double *r)
{
    const int fe = c->opt.restriction == CAMS_R_FE;
    const GridDev &g = c->g;
    const Arrays &a = c->a;
    const int grid = g.Nc;
    if (c->opt.precision == CAMS_MIXED_BF16)
        k_restrict<uint16_t><<<grid, kBlock, 0, c->stream>>>(g, a.dmask, a.Pbf, fe, r, a.slots, a.ictl);
    else if (c->opt.precision == CAMS_MIXED_FP32)
        k_restrict<float><<<grid, kBlock, 0, c->stream>>>(g, a.dmask, a.P32, fe, r, a.slots, a.ictl);
    else
        k_restrict<double><<<grid, kBlock, 0, c->stream>>>(g, a.dmask, a.P, fe, r, a.slots, a.ictl);
}

void launch_batch_residual(const BatchLaunch &L, int par, bool mixed, bool pre)
{
    if (mixed && pre)
        launch_persistent(kb_residual<float, 2>, kBlock, L, L.inst, L.work, L.nwork, par);
    else if (mixed)
        launch_persistent(kb_residual<float, 1>, kBlock, L, L.inst, L.work, L.nwork, par);
    else if (pre)
        launch_persistent(kb_residual<double, 2>, kBlock, L, L.inst, L.work, L.nwork, par);
    else
        launch_persistent(kb_residual<double, 1>, kBlock, L, L.inst, L.work, L.nwork, par);
}

void launch_batch_finalize(const InstDev *inst, int count, hipStream_t st)
{
    kb_finalize<<<count, kFinal, 0, st>>>(inst);
}

void launch_batch_restrict(const BatchLaunch &L, int precision)
{
    if (precision == CAMS_MIXED_BF16)
        launch_persistent(kb_restrict<uint16_t>, kBlock, L, L.inst, L.work, L.nwork);
    else if (precision == CAMS_MIXED_FP32)
        launch_persistent(kb_restrict<float>, kBlock, L, L.inst, L.work, L.nwork);
    else
        launch_persistent(kb_restrict<double>, kBlock, L, L.inst, L.work, L.nwork);
}

void launch_batch_reset(const BatchLaunch &L)
{
    launch_persistent(kb_reset, kBlock, L, L.inst, L.work, L.nwork);
}

void launch_batch_gather(const InstDev *inst, int count, BatchResult *out, hipStream_t st)
{
    kb_gather<<<(count + kBlock - 1) / kBlock, kBlock, 0, st>>>(inst, count, out);
}

}  // namespace cams
