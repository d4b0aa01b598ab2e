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

// v0 + (v1 + v2 + v3 once `fold` is set); the pending corrections are FP64
// or, in the mixed-precision solve, FP32.
template <class TA>
struct Pending {
    const double *v0;
    const TA *v1, *v2, *v3;
    bool fold;
    __device__ __forceinline__ double operator()(int m) const
    {
        double s = v0[m];
        if (fold) {
            if (v1) s += (double)v1[m];
            if (v2) s += (double)v2[m];
            if (v3) s += (double)v3[m];
        }
        return s;
    }
};

// r = r0 - A v over the cells of workgroup `blk` (and its FP32 copy rf when
// given), dp_out = v, and the workgroup's partial of ||r||^2.
template <class TA>
__device__ __forceinline__ void residual_body(const GridDev &g, const double *__restrict__ W,
                                              const double *__restrict__ diag, const double *__restrict__ r0,
                                              const Pending<TA> &v, double *__restrict__ dp_out,
                                              double *__restrict__ r, float *__restrict__ rf,
                                              double *__restrict__ partial, int blk, double *sh)
{
    const int n = blk * kBlock + threadIdx.x;
    double e2 = 0.0;
    if (n < g.N) {
        const Cell c = cell_of(g, n);
        const double *Wx = W, *Wy = W + g.N, *Wz = W + 2 * g.N;
        const double vn = v(n);
        double s = diag[n] * vn;
        if (c.i > 0) s -= Wx[n - 1] * v(n - 1);
        if (c.i + 1 < g.nx) s -= Wx[n] * v(n + 1);
        if (c.j > 0) s -= Wy[n - g.nx] * v(n - g.nx);
        if (c.j + 1 < g.ny) s -= Wy[n] * v(n + g.nx);
        if (c.k > 0) s -= Wz[n - g.sxy] * v(n - g.sxy);
        if (c.k + 1 < g.nz) s -= Wz[n] * v(n + g.sxy);
        const double rr = r0[n] - s;
        r[n] = rr;
        if (rf) rf[n] = (float)rr;
        dp_out[n] = vn;
        e2 = rr * rr;
    }
    const double bs = block_sum<kBlock>(e2, sh);
    if (threadIdx.x == 0) partial[blk] = bs;
}

template <class TA>
__global__ __launch_bounds__(kBlock) void k_residual_ctl(GridDev g, const double *__restrict__ W,
                                                          const double *__restrict__ diag,
                                                          const double *__restrict__ r0, Pending<TA> v,
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

// ||r||^2 from the residual kernel's partials and the stopping test, by one
// workgroup of kFinal threads.
constexpr int kFinal = 1024;

__device__ __forceinline__ void finalize_body(const double *__restrict__ partial, int nparts, int32_t *ictl,
                                              double *scal, double rtol2, int maxit, double *sh)
{
    double u = 0.0;
    for (int t = threadIdx.x; t < nparts; t += kFinal) u += partial[t];
    const double s = block_sum<kFinal>(u, sh);
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

__global__ __launch_bounds__(kFinal) void k_finalize_ctl(const double *__restrict__ partial, int nparts,
                                                          int32_t *ictl, double *scal, double rtol2, int maxit)
{
    __shared__ double sh[kFinal / 64];
    if (ictl[C_DONE]) return;
    finalize_body(partial, nparts, ictl, scal, rtol2, maxit, sh);
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
    const int x0 = g.ob[0][ka], y0 = g.ob[1][kb], z0 = g.ob[2][kc];
    const int ex = g.ob[0][ka + 1] - x0, ey = g.ob[1][kb + 1] - y0, ez = g.ob[2][kc + 1] - z0;
    const int m = ex * ey * ez;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < m; t += kBlock) {
        const int x = x0 + t % ex, y = y0 + (t / ex) % ey, z = z0 + t / (ex * ey);
        const int n = x + g.nx * (y + g.ny * z);
        const double rn = r[n];
        if (fe) {
            if (!dm[n]) {
#pragma unroll
                for (int q = 0; q < 8; ++q) acc[q] += basis_value(P, (size_t)q * g.N + n) * rn;
            }
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

// ---- batched forms: one launch covers every instance of a batch; the work
// item of a workgroup names the instance and the block within it, and
// workgroups of instances that have converged return at once.

template <class TA>
__device__ __forceinline__ Pending<TA> pending_of(const InstDev &d, int par, bool fold);

// Corrections of the previous iteration: d0 (pre-smoothing), then d2, which
// the post-smoothing started from d1 and so holds d1 + d2, or d1 alone
// without post-smoothing.
template <>
__device__ __forceinline__ Pending<double> pending_of<double>(const InstDev &d, int par, bool fold)
{
    return Pending<double>{d.a.dp[par], d.n_pre > 0 ? d.a.d0 : nullptr, d.n_post > 0 ? d.a.d2 : d.a.d1, nullptr,
                           fold};
}

template <>
__device__ __forceinline__ Pending<float> pending_of<float>(const InstDev &d, int par, bool fold)
{
    return Pending<float>{d.a.dp[par], d.n_pre > 0 ? d.a.d0f : nullptr, d.n_post > 0 ? d.a.d2f : d.a.d1f, nullptr,
                          fold};
}

template <class TA>
__global__ __launch_bounds__(kBlock) void kb_residual(const InstDev *__restrict__ inst,
                                                       const WorkItem *__restrict__ work, const int32_t *nwork, int par)
{
    __shared__ double sh[kBlock / 64];
    CAMS_FOR_ITEMS(t, nwork)
    {
        const WorkItem w = work[t];
        const InstDev &d = inst[w.inst];
        if (d.a.ictl[C_DONE]) continue;
        const Pending<TA> v = pending_of<TA>(d, par, d.a.ictl[C_IT] > 0);
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
    finalize_body(d.a.partial, d.nparts, d.a.ictl, d.a.scal, d.rtol2, d.maxit, sh);
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

void launch_residual_ctl(cams_ctx *c, const double *dp_in, const double *a0, const double *a1, const double *a2,
                         double *dp_out)
{
    Pending<double> v{dp_in, a0, a1, a2, false};
    k_residual_ctl<double><<<(c->g.N + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(
        c->g, c->a.W, c->a.diag, c->a.r0, v, dp_out, c->a.r, nullptr, c->a.partial, c->a.ictl);
}

void launch_residual_ctl32(cams_ctx *c, const double *dp_in, const float *a0, const float *a1, const float *a2,
                           double *dp_out, float *rf)
{
    Pending<float> v{dp_in, a0, a1, a2, false};
    k_residual_ctl<float><<<(c->g.N + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(
        c->g, c->a.W, c->a.diag, c->a.r0, v, dp_out, c->a.r, rf, c->a.partial, c->a.ictl);
}

void launch_finalize_ctl(cams_ctx *c)
{
    const double rt = c->opt.lin_rtol;
    k_finalize_ctl<<<1, kFinal, 0, c->stream>>>(c->a.partial, (c->g.N + kBlock - 1) / kBlock, c->a.ictl, c->a.scal,
                                                rt * rt, c->opt.lin_maxit);
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

void launch_batch_residual(const BatchLaunch &L, int par, bool mixed)
{
    if (mixed)
        launch_persistent(kb_residual<float>, kBlock, L, L.inst, L.work, L.nwork, par);
    else
        launch_persistent(kb_residual<double>, kBlock, L, L.inst, L.work, L.nwork, par);
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
