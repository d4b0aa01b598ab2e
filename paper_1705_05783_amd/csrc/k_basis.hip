// Basis functions of type B4 (Sec. 3, Eq. (11)) with reduced-problem
// boundary conditions, built dual region by dual region in wirebasket order:
// vertices (unit value), then dual edge segments, face patches and interior
// boxes.  A region is a box of cells with `nfree` open axes; its local matrix
// keeps the two-point couplings along the open axes only (couplings to the
// lower-dimensional neighbours across a fixed axis are lumped away) and
// takes the already computed values of the higher-dimensional neighbours as
// Dirichlet data.  Each region is solved exactly by one workgroup with a
// banded Cholesky factorisation held in LDS (bandwidth = stride of the last
// open axis: 1 for edges, <= 7 for faces, <= 49 for interiors at ratio 8);
// the up to eight right-hand sides are the region's bracketing coarse nodes.
#include "cams_internal.h"
#include "dev_util.h"

namespace cams {

namespace {

__global__ __launch_bounds__(kBlock) void k_basis_vertices(GridDev g, double *__restrict__ P)
{
    int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    Cell c = cell_of(g, n);
    int lev = g.isv[0][c.i] + g.isv[1][c.j] + (g.dim == 3 ? g.isv[2][c.k] : 0);
#pragma unroll
    for (int s = 0; s < 8; ++s) P[(size_t)s * g.N + n] = (s == 0 && lev == g.dim) ? 1.0 : 0.0;
}

// Blocked banded Cholesky: columns are taken KB at a time.  The first wave
// factors the panel (the KB columns with the <= bw rows below them) with one
// row per lane in registers, pivots and multipliers broadcast by readlane;
// then all threads subtract the panel's rank-KB product from the trailing
// band.  Two barriers per KB columns instead of three per column.
constexpr int KB = 8;

__device__ __forceinline__ double lane_bcast(double v, int lane)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The local system of one region: band of L by columns (L[c*ld + d] = entry
// (c+d, c), ld = bw + 1; once factored, the diagonal entry holds its
// reciprocal) followed by 8 right-hand sides per cell, in dynamic LDS of
// `cap` doubles (sized by the host for the largest region of the stage).
template <int NT>
__device__ __forceinline__ void basis_region_body(const GridDev &g, const double *__restrict__ T,
                                                  const double *__restrict__ adiag, const Region R,
                                                  double *__restrict__ P, int32_t *status, int cap)
{
    extern __shared__ double lds[];
    const int e0 = R.len[0], e1 = R.len[1], e2 = R.len[2];
    const int m = e0 * e1 * e2;
    const int lstride[3] = {1, e0, e0 * e1};
    const int gstride[3] = {1, g.nx, g.sxy};
    int bw = 1;
    for (int a = 0; a < 3; ++a)
        if (R.freemask & (1 << a)) bw = lstride[a];
    const int ld = bw + 1;
    if (m * (ld + 8) > cap || bw + KB > 64) {  // region larger than the launch's buffer: host bug
        if (threadIdx.x == 0) atomicOr(status, F_BAD_INPUT);
        return;
    }
    double *L = lds;
    double *B = lds + m * ld;
    // entry (c + d, c) of the band, or 0 when `ok` is false: read from a
    // clamped in-band address and zeroed afterwards, so that the reads of an
    // unrolled loop need no branches around them
    auto band = [&](int c, int d, bool ok) -> double {
        const double v = L[min(c, m - 1) * ld + min(max(d, 0), bw)];
        return ok ? v : 0.0;
    };
    auto rhs = [&](int i, int q, bool ok) -> double {
        const double v = B[min(max(i, 0), m - 1) * 8 + q];
        return ok ? v : 0.0;
    };
    const int rlo[3] = {g.lo[0][R.s[0]], g.lo[1][R.s[1]], g.lo[2][R.s[2]]};
    const double *Tax[3] = {T, T + g.N, T + 2 * g.N};
    const int ncoord[3] = {g.nx, g.ny, g.nz};

    for (int t = threadIdx.x; t < m * ld; t += NT) L[t] = 0.0;
    for (int t = threadIdx.x; t < m * 8; t += NT) B[t] = 0.0;
    __syncthreads();

    // assemble the local matrix and the Dirichlet data of the boundary.  All
    // loads of a cell go out before the first is used: the couplings of its
    // six faces, the basis values of the neighbours across the faces that
    // leave the region, and their lower vertex indices, from in-range
    // addresses (the cell itself stands in where a face has none); the sums
    // then run in the same order as face by face.
    for (int c = threadIdx.x; c < m; c += NT) {
        const int lc[3] = {c % e0, (c / e0) % e1, c / (e0 * e1)};
        const int x[3] = {R.s[0] + lc[0], R.s[1] + lc[1], R.s[2] + lc[2]};
        const int n = x[0] + g.nx * (x[1] + g.ny * x[2]);
        double tf[6], wv[6][8];
        int lo_nb[6];
        bool face[6], ext[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) {   // face f: axis f / 2, towards -1 (f even) or +1 (f odd)
            const int a = f >> 1, dir = (f & 1) ? 1 : -1;
            const int xa = x[a] + dir;
            face[f] = (R.freemask & (1 << a)) && xa >= 0 && xa < ncoord[a];
            ext[f] = face[f] && !(xa >= R.s[a] && xa < R.s[a] + R.len[a]);
            tf[f] = Tax[a][face[f] && dir < 0 ? n - gstride[a] : n];
            const int nb = ext[f] ? n + dir * gstride[a] : n;
#pragma unroll
            for (int s = 0; s < 8; ++s) wv[f][s] = P[(size_t)s * g.N + nb];
            lo_nb[f] = g.lo[a][ext[f] ? xa : x[a]];
        }
        double dsum = 0.0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            if (!face[f]) continue;
            const int a = f >> 1;
            const double t = tf[f];
            dsum += t;
            if (!ext[f]) {
                if (f & 1) L[c * ld + lstride[a]] = -t;
                continue;
            }
            // neighbour on a higher-level dual entity: known values
            int nlo[3] = {rlo[0], rlo[1], rlo[2]};
            nlo[a] = lo_nb[f];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const double w = wv[f][s];
                if (w == 0.0) continue;
                const int bx = nlo[0] + (s & 1) - rlo[0];
                const int by = nlo[1] + ((s >> 1) & 1) - rlo[1];
                const int bz = nlo[2] + ((s >> 2) & 1) - rlo[2];
                if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) {
                    atomicOr(status, F_BAD_INPUT);
                    continue;
                }
                B[c * 8 + bx + 2 * by + 4 * bz] += t * w;
            }
        }
        L[c * ld] = adiag ? dsum + adiag[n] : dsum;   // B1 / B3: accumulation term on the diagonal
    }
    __syncthreads();

    const int lane = threadIdx.x;   // meaningful in the first wave
    for (int c0 = 0; c0 < m; c0 += KB) {
        const int kc = min(KB, m - c0), nr = min(bw, m - c0 - kc), rows = kc + nr;
        if (threadIdx.x < 64) {
            // panel: lane = row c0 + lane, v[q] = entry (row, c0 + q) inside the band
            double v[KB];
            const int i = c0 + lane;
#pragma unroll
            for (int q = 0; q < KB; ++q) {
                const int d = i - (c0 + q);
                v[q] = band(c0 + q, d, q < kc && lane < rows && d >= 0 && d <= bw);
            }
            bool bad = false;
            double rsv[KB];   // 1 / L(c0 + q, c0 + q), the diagonal as stored
#pragma unroll
            for (int q0 = 0; q0 < KB; ++q0) {
                rsv[q0] = 1.0;
                if (q0 >= kc) break;
                double piv = lane_bcast(v[q0], q0);
                if (!(piv > 0.0)) {
                    bad = true;
                    piv = 1.0;
                }
                const double sq = sqrt(piv);
                const double rs = 1.0 / sq;   // one division per column; the multipliers scale by it
                rsv[q0] = rs;
                v[q0] = lane == q0 ? sq : (lane > q0 ? v[q0] * rs : v[q0]);
#pragma unroll
                for (int q2 = q0 + 1; q2 < KB; ++q2) {
                    if (q2 >= kc) break;
                    const double l = lane_bcast(v[q0], q2);
                    if (lane >= q2) v[q2] -= v[q0] * l;
                }
            }
#pragma unroll
            for (int q = 0; q < KB; ++q) {
                const int d = i - (c0 + q);
                if (q < kc && lane < rows && d >= 0 && d <= bw) L[(c0 + q) * ld + d] = d == 0 ? rsv[q] : v[q];
            }
            if (bad && lane == 0) atomicOr(status, F_BAD_PIVOT);
        }
        __syncthreads();
        // trailing band: entry (i, j), c0 + kc <= j <= i < c0 + kc + nr, minus the
        // panel's products.  Thread: column jj = t % 64 of the trailing block
        // (nr <= bw < 64) with its KB panel values in registers, rows
        // ii = jj + t / 64, + NT / 64, ... (each entry written by one thread);
        // a row's KB panel values are read together, zero outside the band,
        // and summed in column order.
        {
            constexpr int NG = NT / 64;
            const int jj = threadIdx.x & 63;
            if (jj < nr) {
                const int j = c0 + kc + jj;
                double pj[KB];
#pragma unroll
                for (int q = 0; q < KB; ++q) {
                    const int dj = j - (c0 + q);
                    pj[q] = band(c0 + q, dj, q < kc && dj <= bw);
                }
                const int iimax = min(nr - 1, jj + bw);
                // RC rows at a time: their reads go out before any of their
                // writes (which the compiler cannot tell apart from the reads)
                constexpr int RC = 4;
                for (int ii0 = jj + (int)(threadIdx.x >> 6); ii0 <= iimax; ii0 += RC * NG) {
                    double acc[RC];
#pragma unroll
                    for (int u = 0; u < RC; ++u) {
                        const int i = c0 + kc + ii0 + u * NG;
                        const bool row = ii0 + u * NG <= iimax;
                        double a = 0.0;
#pragma unroll
                        for (int q = 0; q < KB; ++q) {
                            const int di = i - (c0 + q);
                            const bool ok = row && q < kc && di <= bw;
                            a += band(c0 + q, di, ok) * pj[q];
                        }
                        acc[u] = a;
                    }
#pragma unroll
                    for (int u = 0; u < RC; ++u) {
                        const int i = c0 + kc + ii0 + u * NG;
                        if (ii0 + u * NG <= iimax) L[j * ld + (i - j)] -= acc[u];
                    }
                }
            }
        }
        __syncthreads();
    }
    // forward substitution L y = b, KB rows at a time: the first 8 lanes solve
    // the diagonal block (one right-hand side each) with the block's factor
    // entries and right-hand sides read into registers first, so the
    // recurrence runs on registers rather than through a chain of LDS reads;
    // then all threads update the <= bw rows below
    for (int c0 = 0; c0 < m; c0 += KB) {
        const int kc = min(KB, m - c0), nr = min(bw, m - c0 - kc);
        if (threadIdx.x < 8) {
            const int q = threadIdx.x;
            double y[KB], Lb[KB][KB];
#pragma unroll
            for (int r = 0; r < KB; ++r) {
                y[r] = rhs(c0 + r, q, r < kc);
#pragma unroll
                for (int c = 0; c <= r; ++c)   // entry (c0 + r, c0 + c), zero outside the band
                    Lb[r][c] = band(c0 + c, r - c, r < kc && r - c <= bw);
            }
#pragma unroll
            for (int r = 0; r < KB; ++r) {
                if (r >= kc) break;
                double s = y[r];
#pragma unroll
                for (int c = 0; c < r; ++c) s -= Lb[r][c] * y[c];
                y[r] = s * Lb[r][r];   // the diagonal is stored inverted
            }
#pragma unroll
            for (int r = 0; r < KB; ++r)
                if (r < kc) B[(c0 + r) * 8 + q] = y[r];
        }
        __syncthreads();
        for (int t0 = threadIdx.x; t0 < nr * 8; t0 += 2 * NT) {   // two entries' reads before their writes
            double acc[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int t = t0 + h * NT;
                const int i = c0 + kc + t / 8, q = t % 8;
                double a = 0.0;
#pragma unroll
                for (int u = 0; u < KB; ++u) {   // columns c0 + u of the block inside the band, in order
                    const int c = c0 + u;
                    const bool ok = t < nr * 8 && u < kc && i - c <= bw;
                    a += band(c, i - c, ok) * rhs(c, q, ok);
                }
                acc[h] = a;
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int t = t0 + h * NT;
                if (t < nr * 8) B[(c0 + kc + t / 8) * 8 + t % 8] -= acc[h];
            }
        }
        __syncthreads();
    }
    // backward substitution L^T x = y, blocks in reverse: the diagonal block,
    // then the <= bw rows above it
    for (int c0 = ((m - 1) / KB) * KB; c0 >= 0; c0 -= KB) {
        const int kc = min(KB, m - c0);
        if (threadIdx.x < 8) {
            const int q = threadIdx.x;
            double x[KB], Lb[KB][KB];
#pragma unroll
            for (int r = 0; r < KB; ++r) {
                x[r] = rhs(c0 + r, q, r < kc);
#pragma unroll
                for (int i = r; i < KB; ++i)   // entry (c0 + i, c0 + r) of L, zero outside the band
                    Lb[r][i] = band(c0 + r, i - r, i < kc && i - r <= bw);
            }
#pragma unroll
            for (int r = KB - 1; r >= 0; --r) {
                if (r >= kc) continue;
                double s = x[r];
#pragma unroll
                for (int i = r + 1; i < KB; ++i) s -= Lb[r][i] * x[i];
                x[r] = s * Lb[r][r];
            }
#pragma unroll
            for (int r = 0; r < KB; ++r)
                if (r < kc) B[(c0 + r) * 8 + q] = x[r];
        }
        __syncthreads();
        const int lo = max(0, c0 - bw), na = c0 - lo;
        for (int t0 = threadIdx.x; t0 < na * 8; t0 += 2 * NT) {
            double acc[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int t = t0 + h * NT;
                const int c = lo + t / 8, q = t % 8;
                double a = 0.0;
#pragma unroll
                for (int u = 0; u < KB; ++u) {   // rows c0 + u of the block inside the band, in order
                    const int i = c0 + u;
                    const bool ok = t < na * 8 && u < kc && i - c <= bw;
                    a += band(c, i - c, ok) * rhs(i, q, ok);
                }
                acc[h] = a;
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int t = t0 + h * NT;
                if (t < na * 8) B[(lo + t / 8) * 8 + t % 8] -= acc[h];
            }
        }
        __syncthreads();
    }
    for (int c = threadIdx.x; c < m; c += NT) {
        const int x0 = R.s[0] + c % e0, x1 = R.s[1] + (c / e0) % e1, x2 = R.s[2] + c / (e0 * e1);
        const int n = x0 + g.nx * (x1 + g.ny * x2);
#pragma unroll
        for (int s = 0; s < 8; ++s) P[(size_t)s * g.N + n] = B[c * 8 + s];
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_basis_region(GridDev g, const double *__restrict__ T,
                                                      const double *__restrict__ adiag,
                                                      const Region *__restrict__ regs, double *__restrict__ P,
                                                      int32_t *status, int cap)
{
    basis_region_body<NT>(g, T, adiag, regs[blockIdx.x], P, status, cap);
}

// The same over the regions of many instances (B4: couplings T, no extra
// diagonal): work item (instance, index into that instance's regions).
template <int NT>
__global__ __launch_bounds__(NT) void kb_basis_region(const InstDev *__restrict__ inst,
                                                       const WorkItem *__restrict__ items, int cap)
{
    const WorkItem w = items[blockIdx.x];
    const InstDev &d = inst[w.inst];
    basis_region_body<NT>(d.g, d.a.T, nullptr, d.a.regions[w.blk], d.a.P, d.a.status, cap);
}

// Couplings and extra diagonal of the local problems of the basis types
// other than B4: B1/B2 couplings T (rho_i + rho_j)/2 at the iterate p (no
// Dirichlet masking); B1 diagonal phi c rho(p^n) dV / dt, B3 phi c dV / dt.
__global__ __launch_bounds__(kBlock) void k_basis_coeffs(GridDev g, Fluid f, const double *__restrict__ T,
                                                          const double *__restrict__ phi,
                                                          const double *__restrict__ p,
                                                          const double *__restrict__ pn, int kind,
                                                          double *__restrict__ C, double *__restrict__ A)
{
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    if (kind == CAMS_BASIS_B1 || kind == CAMS_BASIS_B2) {
        const Cell c = cell_of(g, n);
        const double rho = f.rho0 * exp(f.c * (p[n] - f.p0));
        auto w = [&](int m, double t) { return t * 0.5 * (rho + f.rho0 * exp(f.c * (p[m] - f.p0))); };
        C[n] = c.i + 1 < g.nx ? w(n + 1, T[n]) : 0.0;
        C[g.N + n] = c.j + 1 < g.ny ? w(n + g.nx, T[g.N + n]) : 0.0;
        C[2 * (size_t)g.N + n] = c.k + 1 < g.nz ? w(n + g.sxy, T[2 * (size_t)g.N + n]) : 0.0;
    }
    if (kind == CAMS_BASIS_B1) A[n] = phi[n] * f.c * f.rho0 * exp(f.c * (pn[n] - f.p0)) * g.dV / f.dt;
    if (kind == CAMS_BASIS_B3) A[n] = phi[n] * f.c * g.dV / f.dt;
}

// The coefficients a region's local problem uses: per cell, the faces along
// its open axes (those to cells of the region and to the higher-level
// neighbours whose values are its Dirichlet data) and, with an extra
// diagonal, the cell's own entry.  Each face is used by one region only.
template <class F>
__device__ __forceinline__ void region_coeffs(const GridDev &g, const Region &R, int t, F &&fn)
{
    const int e0 = R.len[0], e1 = R.len[1];
    const int x[3] = {R.s[0] + t % e0, R.s[1] + (t / e0) % e1, R.s[2] + t / (e0 * e1)};
    const int n = x[0] + g.nx * (x[1] + g.ny * x[2]);
    const int gstride[3] = {1, g.nx, g.sxy};
    const int ncoord[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a) {
        if (!(R.freemask & (1 << a))) continue;
        if (x[a] > 0) fn((size_t)a * g.N + (n - gstride[a]));
        if (x[a] + 1 < ncoord[a]) fn((size_t)a * g.N + n);
    }
    fn((size_t)3 * g.N + n);   // the diagonal entry (index 3N + n)
}

// Largest relative change of a region's coefficients against the snapshot
// taken when the region was last solved; flag[r] = 1 when above tol.
__global__ __launch_bounds__(kBlock) void k_region_change(GridDev g, const double *__restrict__ C,
                                                           const double *__restrict__ A,
                                                           const double *__restrict__ Cs,
                                                           const double *__restrict__ As,
                                                           const Region *__restrict__ regs, double tol,
                                                           int32_t *__restrict__ flag)
{
    __shared__ double sh[kBlock];
    const Region R = regs[blockIdx.x];
    const int m = R.len[0] * R.len[1] * R.len[2];
    double mx = 0.0;
    for (int t = threadIdx.x; t < m; t += kBlock)
        region_coeffs(g, R, t, [&](size_t i) {
            double v, o;
            if (i < (size_t)3 * g.N) {
                v = C[i];
                o = Cs[i];
            } else {
                if (!A) return;
                v = A[i - (size_t)3 * g.N];
                o = As[i - (size_t)3 * g.N];
            }
            const double d = fabs(v - o);
            mx = fmax(mx, o != 0.0 ? d / fabs(o) : (d > 0.0 ? 1e300 : 0.0));
        });
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) flag[blockIdx.x] = sh[0] > tol ? 1 : 0;
}

// Snapshot of the coefficients of the listed (just solved) regions.
__global__ __launch_bounds__(kBlock) void k_region_snapshot(GridDev g, const double *__restrict__ C,
                                                             const double *__restrict__ A,
                                                             double *__restrict__ Cs, double *__restrict__ As,
                                                             const Region *__restrict__ regs)
{
    const Region R = regs[blockIdx.x];
    const int m = R.len[0] * R.len[1] * R.len[2];
    for (int t = threadIdx.x; t < m; t += kBlock)
        region_coeffs(g, R, t, [&](size_t i) {
            if (i < (size_t)3 * g.N)
                Cs[i] = C[i];
            else if (A)
                As[i - (size_t)3 * g.N] = A[i - (size_t)3 * g.N];
        });
}

}  // namespace

// Couplings and extra diagonal of the context's basis type.
static void basis_operator(const cams_ctx *c, const double *&C, const double *&A)
{
    const int kind = c->opt.basis_type;
    C = (kind == CAMS_BASIS_B1 || kind == CAMS_BASIS_B2) ? c->a.bcoef : c->a.T;
    A = (kind == CAMS_BASIS_B1 || kind == CAMS_BASIS_B3) ? c->a.bdiag : nullptr;
}

void launch_basis_coeffs(cams_ctx *c, const double *p, const double *pn)
{
    const int kind = c->opt.basis_type;
    if (kind == CAMS_BASIS_B4) return;
    k_basis_coeffs<<<(c->g.N + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(
        c->g, c->fl, c->a.T, c->a.phi, p, pn, kind, c->a.bcoef, c->a.bdiag);
}

void launch_region_change(cams_ctx *c, int first, int count, double tol)
{
    if (count <= 0) return;
    const double *C, *A;
    basis_operator(c, C, A);
    k_region_change<<<count, kBlock, 0, c->stream>>>(c->g, C, A, c->a.bsnap, c->a.bdsnap, c->a.regions + first, tol,
                                                     c->a.rflag + first);
}

void launch_region_snapshot(cams_ctx *c, const Region *regs, int count)
{
    if (count <= 0) return;
    const double *C, *A;
    basis_operator(c, C, A);
    k_region_snapshot<<<count, kBlock, 0, c->stream>>>(c->g, C, A, c->a.bsnap, c->a.bdsnap, regs);
}

void launch_basis_vertices(cams_ctx *c)
{
    const GridDev &g = c->g;
    k_basis_vertices<<<(g.N + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(g, c->a.P);
}

// Systems of at most kOneWaveLds doubles (every dual edge and face patch,
// interiors up to ratio 5) are solved by one-wave workgroups: the panel
// factorisation and the triangular solves use the first wave only, so the
// other three waves of a 256-thread workgroup would mostly wait, and four
// times as many small regions share a compute unit.
constexpr int kOneWaveLds = 2048;   // 16 KB

// Exact local solves of `count` regions with `nfree` open axes (a subset of
// that stage's regions: the LDS is sized for the stage's largest system).
void launch_basis_regions(cams_ctx *c, int nfree, const Region *regs, int count)
{
    if (count <= 0) return;
    const GridDev &g = c->g;
    const int cap = c->maxm[nfree] * (c->maxbw[nfree] + 1 + 8);
    const size_t bytes = (size_t)cap * sizeof(double);
    const double *C, *A;
    basis_operator(c, C, A);
    if (nfree == 1 || cap <= kOneWaveLds)
        k_basis_region<64><<<count, 64, bytes, c->stream>>>(g, C, A, regs, c->a.P, c->a.status, cap);
    else
        k_basis_region<kBlock><<<count, kBlock, bytes, c->stream>>>(g, C, A, regs, c->a.P, c->a.status, cap);
}

void launch_batch_basis_regions(const InstDev *inst, const WorkItem *items, int count, int nfree, int cap,
                                 hipStream_t st)
{
    if (count <= 0) return;
    const size_t bytes = (size_t)cap * sizeof(double);
    if (nfree == 1 || cap <= kOneWaveLds)
        kb_basis_region<64><<<count, 64, bytes, st>>>(inst, items, cap);
    else
        kb_basis_region<kBlock><<<count, kBlock, bytes, st>>>(inst, items, cap);
}

void launch_basis(cams_ctx *c)
{
    launch_basis_vertices(c);
    for (int nfree = 1; nfree <= c->g.dim; ++nfree)
        launch_basis_regions(c, nfree, c->a.regions + c->regoff[nfree], c->nreg[nfree]);
    if (c->opt.basis_type == CAMS_BASIS_B1 || c->opt.basis_type == CAMS_BASIS_B2)
        launch_region_snapshot(c, c->a.regions + c->regoff[1], c->region_total - c->regoff[1]);
}

}  // namespace cams
