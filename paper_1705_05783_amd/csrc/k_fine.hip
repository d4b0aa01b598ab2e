// Fine-grid kernels of the C-AMS solve: two-point transmissibilities, the
// Newton system assembly (Sec. 2, Eqs. (2)-(6), mass form), the 7-point
// residual, prolongation (Eq. (12)) and the red-black ILU(0) smoother
// (Table "cams" step 6).  One thread per cell, x fastest, so every stencil
// load is a coalesced row access; neighbour rows are served from L2.
#include "cams_internal.h"
#include "dev_util.h"

namespace cams {

namespace {

inline int grid_blocks(int n) { return (n + kBlock - 1) / kBlock; }

__global__ __launch_bounds__(kBlock) void k_fill(double *__restrict__ x, int n, double v)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < n) x[t] = v;
}

// Face conductance of two cells in series: (A/h) * 2 l1 l2 / (l1 + l2).
__global__ __launch_bounds__(kBlock) void k_transmissibility(GridDev g, const double *__restrict__ perm,
                                                              double mu, double *__restrict__ T,
                                                              double *__restrict__ Tb)
{
    int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    Cell c = cell_of(g, n);
    double l = perm[n] / mu;
    double tx = 0.0, ty = 0.0, tz = 0.0;
    if (c.i + 1 < g.nx) {
        double m = perm[n + 1] / mu;
        tx = (g.dy * g.dz / g.dx) * (2.0 * l * m / (l + m));
    }
    if (c.j + 1 < g.ny) {
        double m = perm[n + g.nx] / mu;
        ty = (g.dx * g.dz / g.dy) * (2.0 * l * m / (l + m));
    }
    if (c.k + 1 < g.nz) {
        double m = perm[n + g.sxy] / mu;
        tz = (g.dx * g.dy / g.dz) * (2.0 * l * m / (l + m));
    }
    T[n] = tx;
    T[g.N + n] = ty;
    T[2 * g.N + n] = tz;
    // half-cell transmissibility between the centre and a west / east boundary face
    const double tb = (g.dy * g.dz / g.dx) * 2.0 * l;
    if (c.i == 0) Tb[c.j + g.ny * c.k] = tb;
    if (c.i == g.nx - 1) Tb[(size_t)g.ny * g.nz + c.j + g.ny * c.k] = tb;
}

// Flux through a Dirichlet boundary face of cell (i, j, k), if it has one:
// T_b (rho_i + rho(p_b)) / 2 (p_i - p_b); w receives T_b (rho_i + rho(p_b)) / 2.
__device__ __forceinline__ double boundary_flux(const GridDev &g, const Fluid &f, const FaceBC &bc,
                                                const double *__restrict__ Tb, const Cell &c, double pi,
                                                double rho, double &w)
{
    w = 0.0;
    double fl = 0.0;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        if (!bc.on[side] || c.i != (side ? g.nx - 1 : 0)) continue;
        const double t = Tb[(size_t)side * g.ny * g.nz + c.j + g.ny * c.k];
        const double ws = t * 0.5 * (rho + f.rho0 * exp(f.c * (bc.p[side] - f.p0)));
        w += ws;
        fl += ws * (pi - bc.p[side]);
    }
    return fl;
}

__global__ __launch_bounds__(kBlock) void k_check_rock(int N, const double *__restrict__ perm,
                                                        const double *__restrict__ phi, int32_t *status)
{
    int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    double k = perm[n], f = phi[n];
    bool ok = (k > 0.0) && (k < 1e300) && (f > 0.0) && (f <= 1.0);
    if (!ok) atomicOr(status, F_BAD_INPUT);
}

__device__ __forceinline__ double density(const Fluid &f, double p) { return f.rho0 * exp(f.c * (p - f.p0)); }

// Newton system at p: masked W on the upper faces, diagonal, r = -F and the
// per-workgroup partial sums of eps^2 (Eq. (16)).
__global__ __launch_bounds__(kBlock) void k_assemble(GridDev g, Fluid f, const double *__restrict__ T,
                                                      const double *__restrict__ phi, const double *__restrict__ q,
                                                      const uint8_t *__restrict__ dm, const double *__restrict__ p,
                                                      const double *__restrict__ pn, double *__restrict__ W,
                                                      double *__restrict__ diag, double *__restrict__ r0,
                                                      double *__restrict__ partial, const double *__restrict__ Tb,
                                                      FaceBC bc)
{
    __shared__ double sh[kBlock / 64];
    int n = blockIdx.x * kBlock + threadIdx.x;
    double e2 = 0.0;
    if (n < g.N) {
        Cell c = cell_of(g, n);
        const double *Tx = T, *Ty = T + g.N, *Tz = T + 2 * g.N;
        const double pi = p[n];
        const double rho = density(f, pi);
        const bool di = dm[n] != 0;
        double sumW = 0.0, flux = 0.0;
        auto face = [&](int m, double t) -> double {
            double pm = p[m];
            double w = t * 0.5 * (rho + density(f, pm));
            sumW += w;
            flux += w * (pi - pm);
            return (di || dm[m]) ? 0.0 : w;
        };
        double wx = 0.0, wy = 0.0, wz = 0.0;
        if (c.i > 0) face(n - 1, Tx[n - 1]);
        if (c.i + 1 < g.nx) wx = face(n + 1, Tx[n]);
        if (c.j > 0) face(n - g.nx, Ty[n - g.nx]);
        if (c.j + 1 < g.ny) wy = face(n + g.nx, Ty[n]);
        if (c.k > 0) face(n - g.sxy, Tz[n - g.sxy]);
        if (c.k + 1 < g.nz) wz = face(n + g.sxy, Tz[n]);
        double wb;
        flux += boundary_flux(g, f, bc, Tb, c, pi, rho, wb);
        sumW += wb;
        W[n] = wx;
        W[g.N + n] = wy;
        W[2 * g.N + n] = wz;
        if (di) {
            diag[n] = 1.0;
            r0[n] = 0.0;
        } else {
            const double rhon = density(f, pn[n]);
            diag[n] = phi[n] * f.c * rhon * g.dV / f.dt + sumW;
            double F = phi[n] * g.dV * (rho - rhon) / f.dt + flux;
            if (q) F -= rho * q[n] * g.dV;
            r0[n] = -F;
            double e = F / (rho * g.dV);
            e2 = e * e;
        }
    }
    double s = block_sum<kBlock>(e2, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Partial sums of eps^2 (Eq. (16)) at x = p + dp (dp nullable): the
// residual F of k_assemble at another pressure, with nothing else written.
__global__ __launch_bounds__(kBlock) void k_eps_at(GridDev g, Fluid f, const double *__restrict__ T,
                                                    const double *__restrict__ phi, const double *__restrict__ q,
                                                    const uint8_t *__restrict__ dm, const double *__restrict__ p,
                                                    const double *__restrict__ dp, const double *__restrict__ pn,
                                                    double *__restrict__ partial, const double *__restrict__ Tb,
                                                    FaceBC bc)
{
    __shared__ double sh[kBlock / 64];
    int n = blockIdx.x * kBlock + threadIdx.x;
    double e2 = 0.0;
    if (n < g.N && !dm[n]) {
        Cell c = cell_of(g, n);
        const double *Tx = T, *Ty = T + g.N, *Tz = T + 2 * g.N;
        auto x = [&](int m) { return dp ? p[m] + dp[m] : p[m]; };
        const double xi = x(n);
        const double rho = density(f, xi);
        double flux = 0.0;
        auto face = [&](int m, double t) {
            const double xm = x(m);
            flux += t * 0.5 * (rho + density(f, xm)) * (xi - xm);
        };
        if (c.i > 0) face(n - 1, Tx[n - 1]);
        if (c.i + 1 < g.nx) face(n + 1, Tx[n]);
        if (c.j > 0) face(n - g.nx, Ty[n - g.nx]);
        if (c.j + 1 < g.ny) face(n + g.nx, Ty[n]);
        if (c.k > 0) face(n - g.sxy, Tz[n - g.sxy]);
        if (c.k + 1 < g.nz) face(n + g.sxy, Tz[n]);
        double wb;
        flux += boundary_flux(g, f, bc, Tb, c, xi, rho, wb);
        const double rhon = density(f, pn[n]);
        double F = phi[n] * g.dV * (rho - rhon) / f.dt + flux;
        if (q) F -= rho * q[n] * g.dV;
        const double e = F / (rho * g.dV);
        e2 = e * e;
    }
    double s = block_sum<kBlock>(e2, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Two-point mass fluxes of the Newton system assembled at p, at the updated
// pressure x = p + d: on the face between n and its +x/+y/+z neighbour m,
// T (rho(p_n) + rho(p_m)) / 2 (x_n - x_m), positive from n to m, stored on n.
__global__ __launch_bounds__(kBlock) void k_face_flux(GridDev g, Fluid f, const double *__restrict__ T,
                                                       const double *__restrict__ p, const double *__restrict__ d,
                                                       double *__restrict__ flux)
{
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    Cell c = cell_of(g, n);
    const double rho = density(f, p[n]);
    const double xn = p[n] + d[n];
    auto fl = [&](int m, double t) { return t * 0.5 * (rho + density(f, p[m])) * (xn - (p[m] + d[m])); };
    flux[n] = c.i + 1 < g.nx ? fl(n + 1, T[n]) : 0.0;
    flux[g.N + n] = c.j + 1 < g.ny ? fl(n + g.nx, T[g.N + n]) : 0.0;
    flux[2 * (size_t)g.N + n] = c.k + 1 < g.nz ? fl(n + g.sxy, T[2 * (size_t)g.N + n]) : 0.0;
}

// Deterministic final sum of `n` partials by one workgroup.
__global__ __launch_bounds__(kBlock) void k_reduce(const double *__restrict__ partial, int n, double *__restrict__ out)
{
    __shared__ double sh[kBlock / 64];
    double v = 0.0;
    for (int t = threadIdx.x; t < n; t += kBlock) v += partial[t];
    double s = block_sum<kBlock>(v, sh);
    if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(kBlock) void k_impose_wells(double *__restrict__ p, const int32_t *__restrict__ cell,
                                                          const double *__restrict__ val, int nw)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < nw) p[cell[t]] = val[t];
}

// Apply of the 7-point operator to a vector given as a sum of up to four
// arrays; used by the residual kernel, which also folds the pending
// corrections into the accumulated update.
struct VecSum {
    const double *v0, *v1, *v2, *v3;
    __device__ __forceinline__ double operator()(int m) const
    {
        double s = v0[m];
        if (v1) s += v1[m];
        if (v2) s += v2[m];
        if (v3) s += v3[m];
        return s;
    }
};

template <class V>
__device__ __forceinline__ double apply_A(const GridDev &g, const double *__restrict__ W,
                                          const double *__restrict__ diag, const V &x, int n, double xn)
{
    Cell c = cell_of(g, n);
    const double *Wx = W, *Wy = W + g.N, *Wz = W + 2 * g.N;
    double s = diag[n] * xn;
    if (c.i > 0) s -= Wx[n - 1] * x(n - 1);
    if (c.i + 1 < g.nx) s -= Wx[n] * x(n + 1);
    if (c.j > 0) s -= Wy[n - g.nx] * x(n - g.nx);
    if (c.j + 1 < g.ny) s -= Wy[n] * x(n + g.nx);
    if (c.k > 0) s -= Wz[n - g.sxy] * x(n - g.sxy);
    if (c.k + 1 < g.nz) s -= Wz[n] * x(n + g.sxy);
    return s;
}

struct Vec1 {
    const double *v;
    __device__ __forceinline__ double operator()(int m) const { return v[m]; }
};

// out = b - A x   (out may alias b).  Skipped once `done` (nullable) is set.
__global__ __launch_bounds__(kBlock) void k_stencil_sub(GridDev g, const double *__restrict__ W,
                                                         const double *__restrict__ diag, const double *b,
                                                         const double *__restrict__ x, double *out,
                                                         const int32_t *done)
{
    if (done && *done) return;
    int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    Vec1 xv{x};
    double s = b[n] - apply_A(g, W, diag, xv, n, x[n]);
    out[n] = s;
}

// out[n] = (P_hat xc)[n]: the (up to) eight bracketing coarse nodes of cell n.
__device__ __forceinline__ void prolong_body(const GridDev &g, const double *__restrict__ P,
                                             const uint8_t *__restrict__ dm, const double *__restrict__ xc,
                                             double *__restrict__ out, int n)
{
    const Cell c = cell_of(g, n);
    out[n] = prolong_at(g, P, dm, xc, n, c.i, c.j, c.k);
}

__global__ __launch_bounds__(kBlock) void k_prolong(GridDev g, const double *__restrict__ P,
                                                     const uint8_t *__restrict__ dm, const double *__restrict__ xc,
                                                     double *__restrict__ out, const int32_t *done)
{
    if (done && *done) return;
    int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    prolong_body(g, P, dm, xc, out, n);
}

// ILU(0) of A in red-black order (red = even i+j+k first).  Red rows keep
// their diagonal; a black row's pivot loses W^2/diag of each red neighbour.
// invd holds the inverse pivots.
__global__ __launch_bounds__(kBlock) void k_ilu_setup(GridDev g, const double *__restrict__ W,
                                                       const double *__restrict__ diag, double *__restrict__ invd,
                                                       int32_t *status)
{
    int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    Cell c = cell_of(g, n);
    double d = diag[n];
    if ((c.i + c.j + c.k) & 1) {
        const double *Wx = W, *Wy = W + g.N, *Wz = W + 2 * g.N;
        double w;
        if (c.i > 0) { w = Wx[n - 1]; d -= w * w / diag[n - 1]; }
        if (c.i + 1 < g.nx) { w = Wx[n]; d -= w * w / diag[n + 1]; }
        if (c.j > 0) { w = Wy[n - g.nx]; d -= w * w / diag[n - g.nx]; }
        if (c.j + 1 < g.ny) { w = Wy[n]; d -= w * w / diag[n + g.nx]; }
        if (c.k > 0) { w = Wz[n - g.sxy]; d -= w * w / diag[n - g.sxy]; }
        if (c.k + 1 < g.nz) { w = Wz[n]; d -= w * w / diag[n + g.sxy]; }
    }
    if (!(d > 0.0)) {
        atomicOr(status, F_BAD_PIVOT);
        d = 1.0;
    }
    invd[n] = 1.0 / d;
}

// Forward half of M^{-1} z for black cells: x_b = (z_b + sum W z_r / diag_r) / d_b.
__global__ __launch_bounds__(kBlock) void k_rb_black(GridDev g, const double *__restrict__ W,
                                                      const double *__restrict__ invd, const double *__restrict__ z,
                                                      double *__restrict__ x)
{
    int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    Cell c = cell_of(g, n);
    if (((c.i + c.j + c.k) & 1) == 0) return;
    const double *Wx = W, *Wy = W + g.N, *Wz = W + 2 * g.N;
    double s = z[n];
    if (c.i > 0) s += Wx[n - 1] * z[n - 1] * invd[n - 1];
    if (c.i + 1 < g.nx) s += Wx[n] * z[n + 1] * invd[n + 1];
    if (c.j > 0) s += Wy[n - g.nx] * z[n - g.nx] * invd[n - g.nx];
    if (c.j + 1 < g.ny) s += Wy[n] * z[n + g.nx] * invd[n + g.nx];
    if (c.k > 0) s += Wz[n - g.sxy] * z[n - g.sxy] * invd[n - g.sxy];
    if (c.k + 1 < g.nz) s += Wz[n] * z[n + g.sxy] * invd[n + g.sxy];
    x[n] = s * invd[n];
}

// Backward half for red cells, x_r = (z_r + sum W x_b) / diag_r, and the
// Richardson update e = (first ? 0 : e) + x on every cell.
__global__ __launch_bounds__(kBlock) void k_rb_red(GridDev g, const double *__restrict__ W,
                                                    const double *__restrict__ invd, const double *__restrict__ z,
                                                    const double *__restrict__ x, double *__restrict__ e, int first)
{
    int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    Cell c = cell_of(g, n);
    double xn;
    if ((c.i + c.j + c.k) & 1) {
        xn = x[n];
    } else {
        const double *Wx = W, *Wy = W + g.N, *Wz = W + 2 * g.N;
        double s = z[n];
        if (c.i > 0) s += Wx[n - 1] * x[n - 1];
        if (c.i + 1 < g.nx) s += Wx[n] * x[n + 1];
        if (c.j > 0) s += Wy[n - g.nx] * x[n - g.nx];
        if (c.j + 1 < g.ny) s += Wy[n] * x[n + g.nx];
        if (c.k > 0) s += Wz[n - g.sxy] * x[n - g.sxy];
        if (c.k + 1 < g.nz) s += Wz[n] * x[n + g.sxy];
        xn = s * invd[n];
    }
    e[n] = first ? xn : e[n] + xn;
}

__global__ __launch_bounds__(kBlock) void k_axpy(double *__restrict__ y, const double *__restrict__ x, int n)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < n) y[t] += x[t];
}

// ---- batched forms (FP64 solve): work item = (instance, block of kBlock cells)

__global__ __launch_bounds__(kBlock) void kb_prolong(const InstDev *__restrict__ inst,
                                                      const WorkItem *__restrict__ work, const int32_t *nwork)
{
    CAMS_FOR_ITEMS(t, nwork)
    {
        const InstDev *d;
        const int n = flat_cell(inst, work[t], d);
        if (n >= 0) prolong_body(d->g, d->a.P, d->a.dmask, d->a.xc, d->a.d1, n);
    }
}

// r := r - A d0 after pre-smoothing
__global__ __launch_bounds__(kBlock) void kb_sub_pre(const InstDev *__restrict__ inst,
                                                      const WorkItem *__restrict__ work, const int32_t *nwork)
{
    CAMS_FOR_ITEMS(t, nwork)
    {
        const InstDev *d;
        const int n = flat_cell(inst, work[t], d);
        if (n < 0) continue;
        Vec1 xv{d->a.d0};
        d->a.r[n] -= apply_A(d->g, d->a.W, d->a.diag, xv, n, d->a.d0[n]);
    }
}

// p += dp of the instance's last iteration (read from its own counter); runs
// after the iteration has stopped, so the done flag is not consulted.
__global__ __launch_bounds__(kBlock) void kb_update(const InstDev *__restrict__ inst, const WorkItem *__restrict__ work,
                                                     const int32_t *nwork, double *const *__restrict__ p)
{
    CAMS_FOR_ITEMS(t, nwork)
    {
        const WorkItem w = work[t];
        const InstDev &d = inst[w.inst];
        const int n = w.blk * kBlock + threadIdx.x;
        if (n >= d.g.N) continue;
        const int it = d.a.ictl[C_IT];
        p[w.inst][n] += d.a.dp[(it + 1) & 1][n];
    }
}

}  // namespace

void launch_fill(cams_ctx *c, double *x, int n, double v)
{
    k_fill<<<grid_blocks(n), kBlock, 0, c->stream>>>(x, n, v);
}

void launch_transmissibility(cams_ctx *c, const double *perm)
{
    k_transmissibility<<<grid_blocks(c->g.N), kBlock, 0, c->stream>>>(c->g, perm, c->fl.mu, c->a.T, c->a.Tb);
}

void launch_check_rock(cams_ctx *c, const double *perm, const double *phi)
{
    k_check_rock<<<grid_blocks(c->g.N), kBlock, 0, c->stream>>>(c->g.N, perm, phi, c->a.status);
}

void launch_assemble(cams_ctx *c, const double *p, const double *pn)
{
    k_assemble<<<grid_blocks(c->g.N), kBlock, 0, c->stream>>>(
        c->g, c->fl, c->a.T, c->a.phi, c->has_q ? c->a.q : nullptr, c->a.dmask, p, pn, c->a.W, c->a.diag,
        c->a.r0, c->a.partial, c->a.Tb, c->bc);
}

void launch_reduce(cams_ctx *c, const double *partial, int n, double *out)
{
    k_reduce<<<1, kBlock, 0, c->stream>>>(partial, n, out);
}

void launch_face_flux(cams_ctx *c, const double *p, const double *d, double *flux)
{
    k_face_flux<<<grid_blocks(c->g.N), kBlock, 0, c->stream>>>(c->g, c->fl, c->a.T, p, d, flux);
}

void launch_eps_at(cams_ctx *c, const double *p, const double *dp, const double *pn, double *out)
{
    k_eps_at<<<grid_blocks(c->g.N), kBlock, 0, c->stream>>>(c->g, c->fl, c->a.T, c->a.phi,
                                                            c->has_q ? c->a.q : nullptr, c->a.dmask, p, dp, pn,
                                                            c->a.partial, c->a.Tb, c->bc);
    launch_reduce(c, c->a.partial, grid_blocks(c->g.N), out);
}

void launch_impose_wells(cams_ctx *c, double *p)
{
    if (c->nwells == 0) return;
    k_impose_wells<<<grid_blocks(c->nwells), kBlock, 0, c->stream>>>(p, c->a.wcell, c->a.wp, c->nwells);
}

void launch_stencil_sub(cams_ctx *c, const double *b, const double *x, double *out, const int32_t *done)
{
    k_stencil_sub<<<grid_blocks(c->g.N), kBlock, 0, c->stream>>>(c->g, c->a.W, c->a.diag, b, x, out, done);
}

void launch_prolong(cams_ctx *c, const double *xc, double *out, const int32_t *done)
{
    k_prolong<<<grid_blocks(c->g.N), kBlock, 0, c->stream>>>(c->g, c->a.P, c->a.dmask, xc, out, done);
}

void launch_rb_setup(cams_ctx *c)
{
    k_ilu_setup<<<grid_blocks(c->g.N), kBlock, 0, c->stream>>>(c->g, c->a.W, c->a.diag, c->a.invd, c->a.status);
}

void launch_ilu_setup(cams_ctx *c)
{
    if (c->opt.smoother == CAMS_SMOOTH_RB_ILU0)
        launch_rb_setup(c);
    else if (c->opt.smoother == CAMS_SMOOTH_NAT_ILU0)
        launch_nat_setup(c);
    else
        launch_bilu_setup(c);
}

void launch_smooth(cams_ctx *c, const double *rhs, double *e, int steps, const int32_t *done)
{
    if (c->opt.smoother == CAMS_SMOOTH_RB_ILU0)
        launch_rb_smooth(c, rhs, e, steps);   // the red-black path is host-controlled only
    else if (c->opt.smoother == CAMS_SMOOTH_NAT_ILU0)
        launch_nat_smooth(c, rhs, e, steps);  // so is the natural-order one
    else
        launch_bilu_smooth(c, rhs, e, steps, done);
}

// e = sum of `steps` ILU(0)-preconditioned Richardson steps on A e = rhs,
// starting from e = 0:  e += M^{-1}(rhs - A e).
void launch_rb_smooth(cams_ctx *c, const double *rhs, double *e, int steps)
{
    const int nb = grid_blocks(c->g.N);
    for (int s = 0; s < steps; ++s) {
        const double *z = rhs;
        if (s > 0) {
            k_stencil_sub<<<nb, kBlock, 0, c->stream>>>(c->g, c->a.W, c->a.diag, rhs, e, c->a.z, nullptr);
            z = c->a.z;
        }
        k_rb_black<<<nb, kBlock, 0, c->stream>>>(c->g, c->a.W, c->a.invd, z, c->a.x);
        k_rb_red<<<nb, kBlock, 0, c->stream>>>(c->g, c->a.W, c->a.invd, z, c->a.x, e, s == 0);
    }
}

void launch_axpy(cams_ctx *c, double *y, const double *x, int n)
{
    k_axpy<<<grid_blocks(n), kBlock, 0, c->stream>>>(y, x, n);
}

void launch_batch_update(const BatchLaunch &L, double *const *p)
{
    launch_persistent(kb_update, kBlock, L, L.inst, L.work, L.nwork, p);
}

void launch_batch_prolong64(const BatchLaunch &L)
{
    launch_persistent(kb_prolong, kBlock, L, L.inst, L.work, L.nwork);
}

void launch_batch_sub_pre64(const BatchLaunch &L)
{
    launch_persistent(kb_sub_pre, kBlock, L, L.inst, L.work, L.nwork);
}

}  // namespace cams
