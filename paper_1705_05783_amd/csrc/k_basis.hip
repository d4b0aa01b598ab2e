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

// MAXM / MAXBW bound the local system of this stage; the LDS holds the band
// of L by columns (L[c*(bw+1)+d] = entry (c+d, c)) followed by 8 rhs per cell.
template <int NT, int MAXM, int MAXBW>
__global__ __launch_bounds__(NT) void k_basis_region(GridDev g, const double *__restrict__ T,
                                                      const Region *__restrict__ regs, double *__restrict__ P,
                                                      int32_t *status)
{
    __shared__ double lds[MAXM * (MAXBW + 1) + 8 * MAXM];
    const Region R = regs[blockIdx.x];
    const int e0 = R.len[0], e1 = R.len[1], e2 = R.len[2];
    const int m = e0 * e1 * e2;
    const int lstride[3] = {1, e0, e0 * e1};
    const int gstride[3] = {1, g.nx, g.sxy};
    int bw = 1;
    for (int a = 0; a < 3; ++a)
        if (R.freemask & (1 << a)) bw = lstride[a];
    if (m > MAXM || bw > MAXBW) {  // region larger than this stage's buffers: host bug
        if (threadIdx.x == 0) atomicOr(status, F_BAD_INPUT);
        return;
    }
    const int ld = bw + 1;
    double *L = lds;
    double *B = lds + m * ld;
    const int rlo[3] = {g.lo[0][R.s[0]], g.lo[1][R.s[1]], g.lo[2][R.s[2]]};
    const double *Tax[3] = {T, T + g.N, T + 2 * g.N};
    const int ncoord[3] = {g.nx, g.ny, g.nz};

    for (int t = threadIdx.x; t < m * ld; t += NT) L[t] = 0.0;
    for (int t = threadIdx.x; t < m * 8; t += NT) B[t] = 0.0;
    __syncthreads();

    // assemble the local matrix and the Dirichlet data of the boundary
    for (int c = threadIdx.x; c < m; c += NT) {
        const int lc[3] = {c % e0, (c / e0) % e1, c / (e0 * e1)};
        const int x[3] = {R.s[0] + lc[0], R.s[1] + lc[1], R.s[2] + lc[2]};
        const int n = x[0] + g.nx * (x[1] + g.ny * x[2]);
        double dsum = 0.0;
        for (int a = 0; a < 3; ++a) {
            if (!(R.freemask & (1 << a))) continue;
            for (int dir = -1; dir <= 1; dir += 2) {
                const int xa = x[a] + dir;
                if (xa < 0 || xa >= ncoord[a]) continue;
                const double t = dir > 0 ? Tax[a][n] : Tax[a][n - gstride[a]];
                dsum += t;
                if (xa >= R.s[a] && xa < R.s[a] + R.len[a]) {
                    if (dir > 0) L[c * ld + lstride[a]] = -t;
                    continue;
                }
                // neighbour on a higher-level dual entity: known values
                const int nb = n + dir * gstride[a];
                const int nlo[3] = {a == 0 ? g.lo[0][xa] : rlo[0], a == 1 ? g.lo[1][xa] : rlo[1],
                                    a == 2 ? g.lo[2][xa] : rlo[2]};
                for (int s = 0; s < 8; ++s) {
                    const double w = P[(size_t)s * g.N + nb];
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
        }
        L[c * ld] = dsum;
    }
    __syncthreads();

    // banded Cholesky, right looking, one column per step
    for (int c = 0; c < m; ++c) {
        double piv = L[c * ld];
        if (!(piv > 0.0)) {
            if (threadIdx.x == 0) atomicOr(status, F_BAD_PIVOT);
            piv = 1.0;
        }
        const double s = sqrt(piv);
        __syncthreads();
        for (int d = threadIdx.x; d <= bw; d += NT)
            if (c + d < m) L[c * ld + d] = (d == 0) ? s : L[c * ld + d] / s;
        __syncthreads();
        const int nd = min(bw, m - 1 - c);
        for (int t = threadIdx.x; t < nd * nd; t += NT) {
            const int d1 = t % nd + 1, d2 = t / nd + 1;
            if (d1 > d2) continue;
            const double l2 = L[c * ld + d2];
            if (l2 == 0.0) continue;
            const double l1 = L[c * ld + d1];
            if (l1 == 0.0) continue;
            L[(c + d1) * ld + (d2 - d1)] -= l1 * l2;
        }
        __syncthreads();
    }
    // forward substitution L y = b
    for (int c = 0; c < m; ++c) {
        if (threadIdx.x < 8) B[c * 8 + threadIdx.x] /= L[c * ld];
        __syncthreads();
        const int nd = min(bw, m - 1 - c);
        for (int t = threadIdx.x; t < nd * 8; t += NT) {
            const int d = t / 8 + 1, q = t % 8;
            B[(c + d) * 8 + q] -= L[c * ld + d] * B[c * 8 + q];
        }
        __syncthreads();
    }
    // backward substitution L^T x = y
    for (int c = m - 1; c >= 0; --c) {
        if (threadIdx.x < 8) B[c * 8 + threadIdx.x] /= L[c * ld];
        __syncthreads();
        const int nd = min(bw, c);
        for (int t = threadIdx.x; t < nd * 8; t += NT) {
            const int d = t / 8 + 1, q = t % 8;
            B[(c - d) * 8 + q] -= L[(c - d) * ld + d] * B[c * 8 + q];
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

}  // namespace

void launch_basis_vertices(cams_ctx *c)
{
    const GridDev &g = c->g;
    k_basis_vertices<<<(g.N + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(g, c->a.P);
}

// Exact local solves of `count` regions with `nfree` open axes.
void launch_basis_regions(cams_ctx *c, int nfree, const Region *regs, int count)
{
    if (count <= 0) return;
    const GridDev &g = c->g;
    constexpr int E = kMaxRatio - 1;
    if (nfree == 1)
        k_basis_region<64, E, 1><<<count, 64, 0, c->stream>>>(g, c->a.T, regs, c->a.P, c->a.status);
    else if (nfree == 2)
        k_basis_region<kBlock, E * E, E><<<count, kBlock, 0, c->stream>>>(g, c->a.T, regs, c->a.P, c->a.status);
    else
        k_basis_region<kBlock, E * E * E, E * E><<<count, kBlock, 0, c->stream>>>(g, c->a.T, regs, c->a.P,
                                                                            c->a.status);
}

void launch_basis(cams_ctx *c)
{
    launch_basis_vertices(c);
    for (int nfree = 1; nfree <= c->g.dim; ++nfree)
        launch_basis_regions(c, nfree, c->a.regions + c->regoff[nfree], c->nreg[nfree]);
}

}  // namespace cams
