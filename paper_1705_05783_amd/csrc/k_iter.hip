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

// r = r0 - A v over the cells of workgroup `blk`, dp_out = v, and the
// workgroup's partial of ||r||^2.
template <class TA>
__device__ __forceinline__ void residual_body(const GridDev &g, const double *__restrict__ W,
                                              const double *__restrict__ diag, const double *__restrict__ r0,
                                              const Pending<TA> &v, double *__restrict__ dp_out,
                                              double *__restrict__ r, double *__restrict__ partial, int blk,
                                              double *sh)
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
                                                          double *__restrict__ partial, const int32_t *ictl)
{
    __shared__ double sh[kBlock / 64];
    if (ictl[C_DONE]) return;
    v.fold = ictl[C_IT] > 0;
    residual_body(g, W, diag, r0, v, dp_out, r, partial, blockIdx.x, sh);
}

// ||r||^2 from the residual kernel's partials and the stopping test.
// Returns true (in thread 0) when this call ended the iteration.
__device__ __forceinline__ bool finalize_body(const double *__restrict__ partial, int nparts, int32_t *ictl,
                                              double *scal, double rtol2, int maxit, double *sh)
{
    double u = 0.0;
    for (int t = threadIdx.x; t < nparts; t += kBlock) u += partial[t];
    const double s = block_sum<kBlock>(u, sh);
    if (threadIdx.x != 0) return false;
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
        return false;
    }
    ictl[C_OUTCOME] = outcome;
    ictl[C_DONE] = 1;
    return true;
}

__global__ __launch_bounds__(kBlock) void k_finalize_ctl(const double *__restrict__ partial, int nparts,
                                                          int32_t *ictl, double *scal, double rtol2, int maxit)
{
    __shared__ double sh[kBlock / 64];
    if (ictl[C_DONE]) return;
    finalize_body(partial, nparts, ictl, scal, rtol2, maxit, sh);
}

// Restriction R r (Eq. (13)/(15)): one workgroup per (coarse node, z-plane of
// its row's cells); a row box is at most 15 x 15 cells per plane (MSFE
// support at ratio 8), covered by a 16 x 16 thread tile.  MSFV rows are the
// primal block (weights 1); MSFE rows are the basis support (weights P_hat).
// The coarse solve adds the plane sums of each row in order.
__device__ __forceinline__ void restrict_body(const GridDev &g, const uint8_t *__restrict__ dm,
                                              const double *__restrict__ P, int fe, const double *__restrict__ r,
                                              double *__restrict__ planes, int max_planes, int k, int pz,
                                              double *sh)
{
    const int ka = k % g.nb[0], kb = (k / g.nb[0]) % g.nb[1], kc = k / (g.nb[0] * g.nb[1]);
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        const int idx = a == 0 ? ka : (a == 1 ? kb : kc);
        const int n = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz);
        if (fe) {
            lo[a] = idx > 0 ? g.vc[a][idx - 1] + 1 : 0;
            hi[a] = idx < g.nb[a] - 1 ? g.vc[a][idx + 1] - 1 : n - 1;
        } else {
            lo[a] = idx * g.r[a];
            hi[a] = min((idx + 1) * g.r[a], n) - 1;
        }
    }
    const int nplanes = hi[2] - lo[2] + 1;
    if (pz >= nplanes) {   // rows with fewer planes: the unused partials are zero
        if (threadIdx.x == 0) planes[(size_t)k * max_planes + pz] = 0.0;
        return;
    }
    const int x = lo[0] + (threadIdx.x & 15), y = lo[1] + (threadIdx.x >> 4), z = lo[2] + pz;
    double v = 0.0;
    if (x <= hi[0] && y <= hi[1]) {
        const int n = x + g.nx * (y + g.ny * z);
        if (fe) {
            if (!dm[n]) {
                const int sx = ka - g.lo[0][x], sy = kb - g.lo[1][y], sz = kc - g.lo[2][z];
                if (sx >= 0 && sx <= 1 && sy >= 0 && sy <= 1 && sz >= 0 && sz <= 1)
                    v = P[(size_t)(sx + 2 * sy + 4 * sz) * g.N + n] * r[n];
            }
        } else {
            v = r[n];
        }
    }
    const double s = block_sum<kBlock>(v, sh);
    if (threadIdx.x == 0) planes[(size_t)k * max_planes + pz] = s;
}

__global__ __launch_bounds__(kBlock) void k_restrict_planes(GridDev g, const uint8_t *__restrict__ dm,
                                                             const double *__restrict__ P, int fe,
                                                             const double *__restrict__ r,
                                                             double *__restrict__ planes, int max_planes,
                                                             const int32_t *ictl)
{
    __shared__ double sh[kBlock / 64];
    if (ictl[C_DONE]) return;
    restrict_body(g, dm, P, fe, r, planes, max_planes, blockIdx.x, blockIdx.y, sh);
}

// ---- batched forms: one launch covers every instance of a batch; the work
// item of a workgroup names the instance and the block within it, and
// workgroups of instances that have converged return at once.

template <class TA>
__device__ __forceinline__ Pending<TA> pending_of(const InstDev &d, int par, bool fold);

template <>
__device__ __forceinline__ Pending<double> pending_of<double>(const InstDev &d, int par, bool fold)
{
    return Pending<double>{d.a.dp[par], d.n_pre > 0 ? d.a.d0 : nullptr, d.a.d1, d.n_post > 0 ? d.a.d2 : nullptr,
                           fold};
}

template <>
__device__ __forceinline__ Pending<float> pending_of<float>(const InstDev &d, int par, bool fold)
{
    return Pending<float>{d.a.dp[par], d.n_pre > 0 ? d.a.d0f : nullptr, d.a.d1f, d.n_post > 0 ? d.a.d2f : nullptr,
                          fold};
}

template <class TA>
__global__ __launch_bounds__(kBlock) void kb_residual(const InstDev *__restrict__ inst,
                                                       const WorkItem *__restrict__ work, int par)
{
    __shared__ double sh[kBlock / 64];
    const WorkItem w = work[blockIdx.x];
    const InstDev &d = inst[w.inst];
    if (d.a.ictl[C_DONE]) return;
    const Pending<TA> v = pending_of<TA>(d, par, d.a.ictl[C_IT] > 0);
    residual_body(d.g, d.a.W, d.a.diag, d.a.r0, v, d.a.dp[par ^ 1], d.a.r, d.a.partial, w.blk, sh);
}

// One workgroup per instance; `ndone` counts the instances that have stopped.
__global__ __launch_bounds__(kBlock) void kb_finalize(const InstDev *__restrict__ inst, int32_t *ndone)
{
    __shared__ double sh[kBlock / 64];
    const InstDev &d = inst[blockIdx.x];
    if (d.a.ictl[C_DONE]) return;
    if (finalize_body(d.a.partial, d.nparts, d.a.ictl, d.a.scal, d.rtol2, d.maxit, sh)) atomicAdd(ndone, 1);
}

__global__ __launch_bounds__(kBlock) void kb_restrict(const InstDev *__restrict__ inst,
                                                       const WorkItem *__restrict__ work)
{
    __shared__ double sh[kBlock / 64];
    const WorkItem w = work[blockIdx.x];
    const InstDev &d = inst[w.inst];
    if (d.a.ictl[C_DONE]) return;
    restrict_body(d.g, d.a.dmask, d.a.P, d.fe, d.a.r, d.a.planes, d.max_planes, w.blk / d.max_planes,
                  w.blk % d.max_planes, sh);
}

// Iteration state of every instance back to its start (dp = 0, counters 0);
// work item = (instance, block of kBlock cells).
__global__ __launch_bounds__(kBlock) void kb_reset(const InstDev *__restrict__ inst, const WorkItem *__restrict__ work)
{
    const WorkItem w = work[blockIdx.x];
    const InstDev &d = inst[w.inst];
    const int n = w.blk * kBlock + threadIdx.x;
    if (n < d.g.N) d.a.dp[0][n] = 0.0;
    if (w.blk == 0)
        for (int t = threadIdx.x; t < C_NODE + d.g.Nc; t += kBlock) d.a.ictl[t] = 0;
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
        c->g, c->a.W, c->a.diag, c->a.r0, v, dp_out, c->a.r, c->a.partial, c->a.ictl);
}

void launch_residual_ctl32(cams_ctx *c, const double *dp_in, const float *a0, const float *a1, const float *a2,
                           double *dp_out)
{
    Pending<float> v{dp_in, a0, a1, a2, false};
    k_residual_ctl<float><<<(c->g.N + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(
        c->g, c->a.W, c->a.diag, c->a.r0, v, dp_out, c->a.r, c->a.partial, c->a.ictl);
}

void launch_finalize_ctl(cams_ctx *c)
{
    const double rt = c->opt.lin_rtol;
    k_finalize_ctl<<<1, kBlock, 0, c->stream>>>(c->a.partial, (c->g.N + kBlock - 1) / kBlock, c->a.ictl, c->a.scal,
                                                rt * rt, c->opt.lin_maxit);
}

void launch_restrict_planes(cams_ctx *c, const double *r, const int32_t *)
{
    dim3 grid(c->g.Nc, c->max_planes);
    k_restrict_planes<<<grid, kBlock, 0, c->stream>>>(c->g, c->a.dmask, c->a.P, c->opt.restriction == CAMS_R_FE, r,
                                                      c->a.planes, c->max_planes, c->a.ictl);
}

void launch_batch_residual(const BatchLaunch &L, int par, bool mixed)
{
    if (L.count <= 0) return;
    if (mixed)
        kb_residual<float><<<L.count, kBlock, 0, L.stream>>>(L.inst, L.work, par);
    else
        kb_residual<double><<<L.count, kBlock, 0, L.stream>>>(L.inst, L.work, par);
}

void launch_batch_finalize(const InstDev *inst, int count, int32_t *ndone, hipStream_t st)
{
    kb_finalize<<<count, kBlock, 0, st>>>(inst, ndone);
}

void launch_batch_restrict(const BatchLaunch &L)
{
    if (L.count > 0) kb_restrict<<<L.count, kBlock, 0, L.stream>>>(L.inst, L.work);
}

void launch_batch_reset(const BatchLaunch &L)
{
    if (L.count > 0) kb_reset<<<L.count, kBlock, 0, L.stream>>>(L.inst, L.work);
}

void launch_batch_gather(const InstDev *inst, int count, BatchResult *out, hipStream_t st)
{
    kb_gather<<<(count + kBlock - 1) / kBlock, kBlock, 0, st>>>(inst, count, out);
}

}  // namespace cams
