// Mixed-precision pieces of the C-AMS solve: the smoother, the basis
// storage and the prolongation run in FP32 (basis optionally in bfloat16)
// with FP32 accumulation, while the residual r = r0 - A d, the update d, the
// norms and the coarse solve stay in FP64.  The outer C-AMS iteration on the
// FP64 residual is then an iterative refinement: it converges to the FP64
// solution whenever the low-precision correction contracts the error.
//
// The rounded basis replaces the FP64 one everywhere (the coarse operator and
// the restriction use exactly the prolongation that is applied), so the
// multiscale stage stays a consistent Galerkin / finite-volume projection.
#include "cams_internal.h"
#include "dev_util.h"

namespace cams {

namespace {

inline int blocks_of(size_t n) { return (int)((n + kBlock - 1) / kBlock); }

// float -> bfloat16, round to nearest even (inputs are finite).
__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__global__ __launch_bounds__(kBlock) void k_to_f32(const double *__restrict__ src, float *__restrict__ dst, size_t n)
{
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < n) dst[t] = (float)src[t];
}

__global__ __launch_bounds__(kBlock) void k_round_basis(double *__restrict__ P, float *__restrict__ P32,
                                                         uint16_t *__restrict__ Pbf, size_t n, int bf16)
{
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n) return;
    const float f = (float)P[t];
    if (bf16) {
        const uint16_t b = to_bf16(f);
        Pbf[t] = b;
        P[t] = (double)from_bf16(b);
    } else {
        P32[t] = f;
        P[t] = (double)f;
    }
}

// out = P_hat xc in FP32 (basis stored as float or bfloat16).
template <int BF>
__device__ __forceinline__ void prolong_lo_body(const GridDev &g, const float *__restrict__ P32,
                                                const uint16_t *__restrict__ Pbf, const uint8_t *__restrict__ dm,
                                                const double *__restrict__ xc, float *__restrict__ out, int n)
{
    const Cell c = cell_of(g, n);
    if constexpr (BF)
        out[n] = prolong_at(g, Pbf, dm, xc, n, c.i, c.j, c.k);
    else
        out[n] = prolong_at(g, P32, dm, xc, n, c.i, c.j, c.k);
}

template <int BF>
__global__ __launch_bounds__(kBlock) void k_prolong_lo(GridDev g, const float *__restrict__ P32,
                                                        const uint16_t *__restrict__ Pbf,
                                                        const uint8_t *__restrict__ dm, const double *__restrict__ xc,
                                                        float *__restrict__ out, const int32_t *done)
{
    if (done && *done) return;
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    prolong_lo_body<BF>(g, P32, Pbf, dm, xc, out, n);
}

// r -= A x in FP64 with an FP32 correction x (pre-smoothing update), and the
// FP32 copy rf of the new r.
__device__ __forceinline__ void sub64_lo_body(const GridDev &g, const double *__restrict__ W,
                                              const double *__restrict__ diag, const float *__restrict__ x,
                                              double *__restrict__ r, float *__restrict__ rf, int n)
{
    // neighbours outside the grid: the cell itself with coupling 0 (no branches)
    const Cell c = cell_of(g, n);
    const double *Wx = W, *Wy = W + g.N, *Wz = W + 2 * g.N;
    const bool xm = c.i > 0, xp = c.i + 1 < g.nx, ym = c.j > 0, yp = c.j + 1 < g.ny, zm = c.k > 0, zp = c.k + 1 < g.nz;
    const int nxm = xm ? n - 1 : n, nxp = xp ? n + 1 : n, nym = ym ? n - g.nx : n, nyp = yp ? n + g.nx : n;
    const int nzm = zm ? n - g.sxy : n, nzp = zp ? n + g.sxy : n;
    const double wxm = Wx[nxm], wxp = Wx[n], wym = Wy[nym], wyp = Wy[n], wzm = Wz[nzm], wzp = Wz[n];
    double s = diag[n] * (double)x[n];
    s -= (xm ? wxm : 0.0) * (double)x[nxm];
    s -= (xp ? wxp : 0.0) * (double)x[nxp];
    s -= (ym ? wym : 0.0) * (double)x[nym];
    s -= (yp ? wyp : 0.0) * (double)x[nyp];
    s -= (zm ? wzm : 0.0) * (double)x[nzm];
    s -= (zp ? wzp : 0.0) * (double)x[nzp];
    const double rn = r[n] - s;
    r[n] = rn;
    rf[n] = (float)rn;
}

__global__ __launch_bounds__(kBlock) void k_sub64_lo(GridDev g, const double *__restrict__ W,
                                                      const double *__restrict__ diag, const float *__restrict__ x,
                                                      double *__restrict__ r, float *__restrict__ rf,
                                                      const int32_t *done)
{
    if (done && *done) return;
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    sub64_lo_body(g, W, diag, x, r, rf, n);
}

// ---- batched forms: work item = (instance, block of kBlock cells)

template <int BF>
__global__ __launch_bounds__(kBlock) void kb_prolong_lo(const InstDev *__restrict__ inst,
                                                         const WorkItem *__restrict__ work, const int32_t *nwork)
{
    CAMS_FOR_ITEMS(t, nwork)
    {
        const InstDev *d;
        const int n = flat_cell(inst, work[t], d);
        if (n >= 0) prolong_lo_body<BF>(d->g, d->a.P32, d->a.Pbf, d->a.dmask, d->a.xc, d->a.d1f, n);
    }
}

__global__ __launch_bounds__(kBlock) void kb_sub64_lo(const InstDev *__restrict__ inst,
                                                       const WorkItem *__restrict__ work, const int32_t *nwork)
{
    CAMS_FOR_ITEMS(t, nwork)
    {
        const InstDev *d;
        const int n = flat_cell(inst, work[t], d);
        if (n >= 0) sub64_lo_body(d->g, d->a.W, d->a.diag, d->a.d0f, d->a.r, d->a.r1f, n);
    }
}

}  // namespace

void launch_convert_matrix32(cams_ctx *c)
{
    const size_t n = (size_t)c->g.N;
    k_to_f32<<<blocks_of(3 * n), kBlock, 0, c->stream>>>(c->a.W, c->a.W32, 3 * n);
    k_to_f32<<<blocks_of(n), kBlock, 0, c->stream>>>(c->a.diag, c->a.diag32, n);
    const size_t npiv = c->opt.smoother == CAMS_SMOOTH_BLOCK_ALT_ILU0 ? 2 * n : n;   // both pivot sets
    k_to_f32<<<blocks_of(npiv), kBlock, 0, c->stream>>>(c->a.invd, c->a.invd32, npiv);
}

void launch_round_basis(cams_ctx *c)
{
    const size_t n = (size_t)c->g.N * 8;
    k_round_basis<<<blocks_of(n), kBlock, 0, c->stream>>>(c->a.P, c->a.P32, c->a.Pbf, n,
                                                          c->opt.precision == CAMS_MIXED_BF16);
}

void launch_prolong32(cams_ctx *c, const double *xc, float *out, const int32_t *done)
{
    if (c->opt.precision == CAMS_MIXED_BF16)
        k_prolong_lo<1><<<blocks_of(c->g.N), kBlock, 0, c->stream>>>(c->g, c->a.P32, c->a.Pbf, c->a.dmask, xc, out,
                                                                      done);
    else
        k_prolong_lo<0><<<blocks_of(c->g.N), kBlock, 0, c->stream>>>(c->g, c->a.P32, c->a.Pbf, c->a.dmask, xc, out,
                                                                      done);
}

void launch_sub64_lo(cams_ctx *c, const float *x, double *r, const int32_t *done)
{
    k_sub64_lo<<<blocks_of(c->g.N), kBlock, 0, c->stream>>>(c->g, c->a.W, c->a.diag, x, r, c->a.r1f, done);
}

void launch_batch_prolong(const BatchLaunch &L, bool mixed, bool bf16)
{
    if (!mixed)
        launch_batch_prolong64(L);
    else if (bf16)
        launch_persistent(kb_prolong_lo<1>, kBlock, L, L.inst, L.work, L.nwork);
    else
        launch_persistent(kb_prolong_lo<0>, kBlock, L, L.inst, L.work, L.nwork);
}

void launch_batch_sub_pre(const BatchLaunch &L, bool mixed)
{
    if (mixed)
        launch_persistent(kb_sub64_lo, kBlock, L, L.inst, L.work, L.nwork);
    else
        launch_batch_sub_pre64(L);
}

}  // namespace cams
