// Coarse level of the C-AMS solve (Sec. 3, Eqs. (7), (13)-(15)):
//  - A_c = R A P_hat: MSFE by owner boxes (each cell's stencil and basis
//    read once, 160 sums per box, then the 8 boxes around each node); MSFV
//    one workgroup per coarse row (the rows of the primal block).  Fixed
//    reduction orders, no atomics: A_c is bitwise deterministic.
//  - the explicit inverse, so that every coarse solve of the iteration is one
//    fully parallel GEMV instead of two latency-bound triangular sweeps:
//    MSFE (symmetric positive definite): Gauss-Jordan sweeps over 64-column
//    panels that update the lower triangle only, the products on FP64
//    matrix cores (v_mfma_f64_16x16x4f64, 64x64 tiles per workgroup), the
//    64x64 pivot-block inverse overlapping the next update; MSFV: LU with
//    partial pivoting by panels, then the
//    inverse from the factors with the same kernels.  Large MSFE coarse grids
//    are eliminated plane by plane (block tridiagonal).
//  - the batched MSFE factorisation of many instances (the same Gauss-Jordan
//    sweeps, every instance's step in one launch).
#include "cams_internal.h"
#include "dev_util.h"

#include <algorithm>

namespace cams {

namespace {

constexpr int kNB = 64;   // LU panel width

// ---- MSFE coarse operator A_c = P^T A P by owner boxes (Eq. (13)).  The
// cells of owner box L (the cells whose lower bracketing node is L) share
// their 8 bracketing nodes I = L + s, s in {0,1}^3.  For such a cell i,
// (A P_J)(i) = sum over the stencil points m of A_im P_J(m) is nonzero only
// for J = L + u with u in {0,1}^3 or one coordinate of u in {-1, 2} (the
// nodes of i and of its six neighbours; 32 values), and P_I(i) (A P_J)(i)
// contributes to A_c[I][J] with J - I = d in {-1,0,1}^3.  Stage 1: one
// workgroup per box forms the 160 reachable (s, d) sums over the box's cells
// in a fixed order, boxp[L][27 s + d]; stage 2 adds the
// 8 boxes around each node in a fixed order.  Deterministic; each cell and
// its stencil are read once instead of once per node whose support holds it.
constexpr int kOpThreads = 512;

__device__ __forceinline__ constexpr int u_index(int ux, int uy, int uz) { return (ux + 1) + 4 * (uy + 1) + 16 * (uz + 1); }

__device__ __forceinline__ constexpr bool u_reach(int ux, int uy, int uz)
{
    // at most one coordinate outside {0, 1}, and that one in {-1, 2}
    const int out = (ux < 0 || ux > 1) + (uy < 0 || uy > 1) + (uz < 0 || uz > 1);
    return out <= 1 && ux >= -1 && ux <= 2 && uy >= -1 && uy <= 2 && uz >= -1 && uz <= 2;
}

__global__ __launch_bounds__(kBlock) void k_zero(double *__restrict__ a, size_t n)
{
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < n) a[t] = 0.0;
}

__global__ __launch_bounds__(kOpThreads) void k_coarse_box(GridDev g, const double *__restrict__ W,
                                                            const double *__restrict__ diag,
                                                            const uint8_t *__restrict__ dm,
                                                            const double *__restrict__ P, double *__restrict__ boxp)
{
    // The 160 reachable (s, d) pairs are reduced over the box's cells 16 at
    // a time: every thread writes its cell's 16 products to LDS, then 32
    // threads per pair add 16 cells each in order and combine their partial
    // sums by DPP exchanges within rows of 16 and two lane reads.
    constexpr int CH = 16, NPAIR = 160;
    __shared__ double buf[CH][kOpThreads];
    __shared__ double part[216];
    __shared__ short pair_sd[NPAIR];
    const int L = blockIdx.x;
    const int la = L % g.nb[0], lb = (L / g.nb[0]) % g.nb[1], lc = L / (g.nb[0] * g.nb[1]);
    const int x0 = g.ob[0][la], y0 = g.ob[1][lb], z0 = g.ob[2][lc];
    const int ex = g.ob[0][la + 1] - x0, ey = g.ob[1][lb + 1] - y0, ez = g.ob[2][lc + 1] - z0;
    const int m = ex * ey * ez;
    for (int q = threadIdx.x; q < 216; q += kOpThreads) part[q] = 0.0;
    if (threadIdx.x == 0) {
        int p = 0;
        for (int s = 0; s < 8; ++s)
            for (int d = 0; d < 27; ++d) {
                const int ux = (s & 1) + d % 3 - 1, uy = ((s >> 1) & 1) + (d / 3) % 3 - 1, uz = (s >> 2) + d / 9 - 1;
                if (u_reach(ux, uy, uz)) pair_sd[p++] = (short)(s * 27 + d);
            }
    }
    const double *Wa[3] = {W, W + g.N, W + 2 * g.N};
    const int Lv[3] = {la, lb, lc};
    for (int t0 = 0; t0 < m; t0 += kOpThreads) {   // uniform trip count: every thread takes part in the sums
        const int t = t0 + threadIdx.x;
        const bool act = t < m;
        const int tt = act ? t : 0;
        const int ci[3] = {x0 + tt % ex, y0 + (tt / ex) % ey, z0 + tt / (ex * ey)};
        const int n = ci[0] + g.nx * (ci[1] + g.ny * ci[2]);
        // every load of the cell first (basis of the cell and of its six
        // neighbours, couplings, masks, node tables), so that they are all in
        // flight together; a neighbour outside the grid reads the cell itself
        int nm[6], cm[6];
        bool inside[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int a = f >> 1, dir = (f & 1) ? 1 : -1;
            const int ext = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz);
            const int stride = a == 0 ? 1 : (a == 1 ? g.nx : g.sxy);
            inside[f] = dir < 0 ? ci[a] > 0 : ci[a] + 1 < ext;
            nm[f] = inside[f] ? n + dir * stride : n;
            cm[f] = inside[f] ? ci[a] + dir : ci[a];
        }
        double pc[8], pn[6][8], cf[6];
        uint8_t dmn[6];
        int lon[6];
#pragma unroll
        for (int s = 0; s < 8; ++s) pc[s] = P[(size_t)s * g.N + n];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int a = f >> 1;
#pragma unroll
            for (int s = 0; s < 8; ++s) pn[f][s] = P[(size_t)s * g.N + nm[f]];
            cf[f] = (f & 1) ? Wa[a][n] : Wa[a][nm[f]];
            dmn[f] = dm[nm[f]];
            lon[f] = g.lo[a][cm[f]];
        }
        const double dg = diag[n];
        const bool keep = act && !dm[n];
        __builtin_amdgcn_sched_barrier(0);
        double w[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const bool in = la + (s & 1) < g.nb[0] && lb + ((s >> 1) & 1) < g.nb[1] && lc + (s >> 2) < g.nb[2];
            w[s] = keep && in ? pc[s] : 0.0;
        }
        double v[64];
#pragma unroll
        for (int q = 0; q < 64; ++q) v[q] = 0.0;
#pragma unroll
        for (int s = 0; s < 8; ++s) v[u_index(s & 1, (s >> 1) & 1, s >> 2)] += dg * pc[s];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int a = f >> 1, dir = (f & 1) ? 1 : -1;
            const double coef = -cf[f];
            const bool ok = inside[f] && !dmn[f];
            const bool moved = lon[f] != Lv[a];   // the neighbour's lower node is L + dir e_a
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int t3[3] = {s & 1, (s >> 1) & 1, s >> 2};
                const double val = ok ? coef * pn[f][s] : 0.0;
                int us[3] = {t3[0], t3[1], t3[2]};
                v[u_index(us[0], us[1], us[2])] += moved ? 0.0 : val;
                us[a] += dir;
                v[u_index(us[0], us[1], us[2])] += moved ? val : 0.0;
            }
        }
#pragma unroll
        for (int chunk = 0; chunk < NPAIR / CH; ++chunk) {
            int p = 0;
#pragma unroll
            for (int s = 0; s < 8; ++s)
#pragma unroll
                for (int d = 0; d < 27; ++d) {
                    const int ux = (s & 1) + d % 3 - 1, uy = ((s >> 1) & 1) + (d / 3) % 3 - 1,
                              uz = (s >> 2) + d / 9 - 1;
                    if (!u_reach(ux, uy, uz)) continue;   // resolved at compile time
                    if (p / CH == chunk) buf[p % CH][threadIdx.x] = w[s] * v[u_index(ux, uy, uz)];
                    ++p;
                }
            __syncthreads();
            {
                const int j = threadIdx.x >> 5, l32 = threadIdx.x & 31;
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < kOpThreads / 32; ++k) acc += buf[j][l32 + 32 * k];
                acc += dpp_f64<0xB1>(acc);    // quad_perm [1,0,3,2]
                acc += dpp_f64<0x4E>(acc);    // quad_perm [2,3,0,1]
                acc += dpp_f64<0x141>(acc);   // row_half_mirror
                acc += dpp_f64<0x140>(acc);   // row_mirror
                const double lo = read_lane_f64(acc, 0) + read_lane_f64(acc, 16);
                const double hi = read_lane_f64(acc, 32) + read_lane_f64(acc, 48);
                if (l32 == 0) {
                    const int q = pair_sd[chunk * CH + j];
                    part[q] += (threadIdx.x & 32) ? hi : lo;
                }
            }
            __syncthreads();
        }
    }
    for (int q = threadIdx.x; q < 216; q += kOpThreads) boxp[(size_t)L * 216 + q] = part[q];
}

// A_c[I][I + d] = sum over s of boxp[I - s][27 s + d] (boxes inside the
// grid), s in increasing order; entries outside the 27-point pattern are
// left as they are (zero).
__global__ __launch_bounds__(kBlock) void k_coarse_nodes(GridDev g, const double *__restrict__ boxp,
                                                          double *__restrict__ Ac)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= 27 * g.Nc) return;
    const int I = t / 27, d = t % 27;
    const int ia = I % g.nb[0], ib = (I / g.nb[0]) % g.nb[1], ic = I / (g.nb[0] * g.nb[1]);
    const int ja = ia + d % 3 - 1, jb = ib + (d / 3) % 3 - 1, jc = ic + d / 9 - 1;
    if (ja < 0 || ja >= g.nb[0] || jb < 0 || jb >= g.nb[1] || jc < 0 || jc >= g.nb[2]) return;
    double sum = 0.0;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int la = ia - (s & 1), lb = ib - ((s >> 1) & 1), lc = ic - (s >> 2);
        if (la < 0 || lb < 0 || lc < 0) continue;
        sum += boxp[(size_t)(la + g.nb[0] * (lb + g.nb[1] * lc)) * 216 + s * 27 + d];
    }
    Ac[(size_t)I * g.Nc + (ja + g.nb[0] * (jb + g.nb[1] * jc))] = sum;
}

// Coarse-operator change since the last factorisation: entry t = 27 I + d of
// the 27-point pattern (node I, neighbour offset d) against the snapshot;
// per-workgroup maxima of the relative change, or (snap) the snapshot itself.
__global__ __launch_bounds__(kBlock) void k_coarse_change(GridDev g, const double *__restrict__ Ac,
                                                           double *__restrict__ Acs, int snap,
                                                           double *__restrict__ partial)
{
    __shared__ double sh[kBlock];
    const int t = blockIdx.x * kBlock + threadIdx.x;
    double rel = 0.0;
    if (t < 27 * g.Nc) {
        const int I = t / 27, d = t % 27;
        const int ia = I % g.nb[0], ib = (I / g.nb[0]) % g.nb[1], ic = I / (g.nb[0] * g.nb[1]);
        const int ja = ia + d % 3 - 1, jb = ib + (d / 3) % 3 - 1, jc = ic + d / 9 - 1;
        double v = 0.0;
        if (ja >= 0 && ja < g.nb[0] && jb >= 0 && jb < g.nb[1] && jc >= 0 && jc < g.nb[2])
            v = Ac[(size_t)I * g.Nc + (ja + g.nb[0] * (jb + g.nb[1] * jc))];
        if (snap) {
            Acs[t] = v;
        } else {
            const double o = Acs[t], dv = fabs(v - o);
            rel = o != 0.0 ? dv / fabs(o) : (dv > 0.0 ? 1e300 : 0.0);
        }
    }
    if (snap) return;
    sh[threadIdx.x] = rel;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kBlock) void k_max_reduce(const double *__restrict__ partial, int n,
                                                        double *__restrict__ out)
{
    __shared__ double sh[kBlock];
    double m = 0.0;
    for (int t = threadIdx.x; t < n; t += kBlock) m = fmax(m, partial[t]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// Cell range of coarse row k along one axis.
__device__ __forceinline__ void row_range(const GridDev &g, int axis, int a, int fe, int &lo, int &hi)
{
    const int n = axis == 0 ? g.nx : (axis == 1 ? g.ny : g.nz);
    if (fe) {
        const int32_t *v = g.vc[axis];
        lo = a > 0 ? v[a - 1] + 1 : 0;
        hi = a < g.nb[axis] - 1 ? v[a + 1] - 1 : n - 1;
    } else {
        lo = a * g.r[axis];
        hi = min((a + 1) * g.r[axis], n) - 1;
    }
}

// Row k of A_c: sum over the row's cells of w_i (A P_hat)_{i,l}, with w_i
// the basis value of node k at cell i (MSFE) or 1 (MSFV).
__global__ __launch_bounds__(kBlock) void k_coarse_row(GridDev g, const double *__restrict__ W,
                                                        const double *__restrict__ diag,
                                                        const uint8_t *__restrict__ dm, const double *__restrict__ P,
                                                        int fe, double *__restrict__ Ac)
{
    __shared__ double acc[27][kBlock];
    __shared__ double row[27];
    const int k = blockIdx.x;
    const int ka = k % g.nb[0], kb = (k / g.nb[0]) % g.nb[1], kc = k / (g.nb[0] * g.nb[1]);
    int lo[3], hi[3];
    row_range(g, 0, ka, fe, lo[0], hi[0]);
    row_range(g, 1, kb, fe, lo[1], hi[1]);
    row_range(g, 2, kc, fe, lo[2], hi[2]);
    for (int t = 0; t < 27; ++t) acc[t][threadIdx.x] = 0.0;
    const int ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
    const int cnt = ex * ey * ez;
    const double *Wa[3] = {W, W + g.N, W + 2 * g.N};
    for (int t = threadIdx.x; t < cnt; t += kBlock) {
        const int i = lo[0] + t % ex, j = lo[1] + (t / ex) % ey, kk = lo[2] + t / (ex * ey);
        const int n = i + g.nx * (j + g.ny * kk);
        if (dm[n]) continue;
        double w = 1.0;
        if (fe) {
            const int sx = ka - g.lo[0][i], sy = kb - g.lo[1][j], sz = kc - g.lo[2][kk];
            if (sx < 0 || sx > 1 || sy < 0 || sy > 1 || sz < 0 || sz > 1) continue;
            w = P[(size_t)(sx + 2 * sy + 4 * sz) * g.N + n];
            if (w == 0.0) continue;
        }
        // the seven points of row n of A
        for (int pt = 0; pt < 7; ++pt) {
            int m = n, mi = i, mj = j, mk = kk;
            double coef;
            if (pt == 0) {
                coef = diag[n];
            } else {
                const int a = (pt - 1) >> 1, dir = ((pt - 1) & 1) ? 1 : -1;
                if (a == 0) { mi += dir; if (mi < 0 || mi >= g.nx) continue; m += dir; }
                if (a == 1) { mj += dir; if (mj < 0 || mj >= g.ny) continue; m += dir * g.nx; }
                if (a == 2) { mk += dir; if (mk < 0 || mk >= g.nz) continue; m += dir * g.sxy; }
                coef = -(dir > 0 ? Wa[a][n] : Wa[a][m]);
            }
            if (coef == 0.0 || dm[m]) continue;
            const int la = g.lo[0][mi], lb = g.lo[1][mj], lc = g.lo[2][mk];
            for (int s = 0; s < 8; ++s) {
                const double pw = P[(size_t)s * g.N + m];
                if (pw == 0.0) continue;
                const int ox = la + (s & 1) - ka + 1, oy = lb + ((s >> 1) & 1) - kb + 1,
                          oz = lc + ((s >> 2) & 1) - kc + 1;
                if (ox < 0 || ox > 2 || oy < 0 || oy > 2 || oz < 0 || oz > 2) continue;  // cannot happen
                acc[ox + 3 * oy + 9 * oz][threadIdx.x] += w * coef * pw;
            }
        }
    }
    __syncthreads();
    // fixed-order (serial) reduction of each of the 27 entries over the threads
    for (int e = threadIdx.x; e < 27; e += kBlock) {
        double s = 0.0;
        for (int t = 0; t < kBlock; ++t) s += acc[e][t];
        row[e] = s;
    }
    __syncthreads();
    const size_t base = (size_t)k * g.Nc;
    for (int col = threadIdx.x; col < g.Nc; col += kBlock) {
        const int ca = col % g.nb[0], cb = (col / g.nb[0]) % g.nb[1], cc = col / (g.nb[0] * g.nb[1]);
        const int ox = ca - ka + 1, oy = cb - kb + 1, oz = cc - kc + 1;
        double v = 0.0;
        if (ox >= 0 && ox <= 2 && oy >= 0 && oy <= 2 && oz >= 0 && oz <= 2) v = row[ox + 3 * oy + 9 * oz];
        Ac[base + col] = v;
    }
}

// ---------------------------------------------------------------- LU ----

// Factor columns [j0, j0+nb) of the row-major n x n matrix A (rows j0..n-1):
// partial pivoting inside the panel; interchanges recorded in piv.
__global__ __launch_bounds__(kBlock) void k_lu_panel(double *__restrict__ A, int n, int j0, int nb,
                                                      int32_t *__restrict__ piv, int32_t *status)
{
    __shared__ double sv[kBlock];
    __shared__ int si[kBlock];
    for (int c = j0; c < j0 + nb; ++c) {
        double best = -1.0;
        int bi = c;
        for (int i = c + threadIdx.x; i < n; i += kBlock) {
            const double v = fabs(A[(size_t)i * n + c]);
            if (v > best) { best = v; bi = i; }
        }
        sv[threadIdx.x] = best;
        si[threadIdx.x] = bi;
        __syncthreads();
        for (int off = kBlock / 2; off > 0; off >>= 1) {
            if (threadIdx.x < off) {
                const double o = sv[threadIdx.x + off];
                const int oi = si[threadIdx.x + off];
                if (o > sv[threadIdx.x] || (o == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                    sv[threadIdx.x] = o;
                    si[threadIdx.x] = oi;
                }
            }
            __syncthreads();
        }
        const int p = si[0];
        if (threadIdx.x == 0) {
            piv[c] = p;
            if (!(sv[0] > 0.0)) atomicOr(status, F_SINGULAR_COARSE);
        }
        if (p != c) {
            for (int col = j0 + threadIdx.x; col < j0 + nb; col += kBlock) {
                const double t = A[(size_t)c * n + col];
                A[(size_t)c * n + col] = A[(size_t)p * n + col];
                A[(size_t)p * n + col] = t;
            }
        }
        __syncthreads();
        double pv = A[(size_t)c * n + c];
        if (pv == 0.0) pv = 1.0;  // flagged above; keep the arithmetic finite
        for (int i = c + 1 + threadIdx.x; i < n; i += kBlock) {
            const double l = A[(size_t)i * n + c] / pv;
            A[(size_t)i * n + c] = l;
            if (l != 0.0)
                for (int col = c + 1; col < j0 + nb; ++col) A[(size_t)i * n + col] -= l * A[(size_t)c * n + col];
        }
        __syncthreads();
    }
}

// Same factorisation with the whole panel ((n - j0) x nb, row stride nb + 1
// against bank conflicts, at most kPanelLds doubles) held in LDS: one global
// read and write of the panel.
constexpr int kPanelLds = 16640;   // 256 rows x 65

__global__ __launch_bounds__(kBlock) void k_lu_panel_lds(double *__restrict__ A, int n, int j0, int nb,
                                                          int32_t *__restrict__ piv, int32_t *status)
{
    __shared__ double Ps[kPanelLds];
    __shared__ double wv[kBlock / 64];
    __shared__ int wi[kBlock / 64];
    const int m = n - j0;
    const int ld = nb + 1;
    for (int t = threadIdx.x; t < m * nb; t += kBlock) {
        const int i = t / nb, c = t % nb;
        Ps[i * ld + c] = A[(size_t)(j0 + i) * n + j0 + c];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int cc = 0; cc < nb; ++cc) {
        // pivot: largest |entry| of column cc in rows cc..m-1 (lowest row on ties)
        double best = -1.0;
        int bi = cc;
        for (int i = cc + threadIdx.x; i < m; i += kBlock) {
            const double v = fabs(Ps[i * ld + cc]);
            if (v > best) { best = v; bi = i; }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_down(best, off, 64);
            const int oi = __shfl_down(bi, off, 64);
            if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
        }
        if (lane == 0) { wv[w] = best; wi[w] = bi; }
        __syncthreads();
        double pb = wv[0];
        int p = wi[0];
        for (int t = 1; t < kBlock / 64; ++t)
            if (wv[t] > pb || (wv[t] == pb && wi[t] < p)) { pb = wv[t]; p = wi[t]; }
        if (threadIdx.x == 0) {
            piv[j0 + cc] = j0 + p;
            if (!(pb > 0.0)) atomicOr(status, F_SINGULAR_COARSE);
        }
        if (p != cc)
            for (int c = threadIdx.x; c < nb; c += kBlock) {
                const double t = Ps[cc * ld + c];
                Ps[cc * ld + c] = Ps[p * ld + c];
                Ps[p * ld + c] = t;
            }
        __syncthreads();
        double pv = Ps[cc * ld + cc];
        if (pv == 0.0) pv = 1.0;  // flagged above; keep the arithmetic finite
        for (int i = cc + 1 + threadIdx.x; i < m; i += kBlock) Ps[i * ld + cc] /= pv;
        __syncthreads();
        // rank-1 update: lane = column, waves stride over rows; each chunk of
        // eight rows is read before it is written so the LDS reads overlap
        const int c = cc + 1 + lane;
        if (c < nb) {
            const double u = Ps[cc * ld + c];
            constexpr int RS = kBlock / 64, CH = 8;
            for (int i0 = cc + 1 + w; i0 < m; i0 += RS * CH) {
                double l[CH], v[CH];
#pragma unroll
                for (int q = 0; q < CH; ++q) {
                    const int i = i0 + q * RS;
                    l[q] = i < m ? Ps[i * ld + cc] : 0.0;
                    v[q] = i < m ? Ps[i * ld + c] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < CH; ++q) {
                    const int i = i0 + q * RS;
                    if (i < m) Ps[i * ld + c] = v[q] - l[q] * u;
                }
            }
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < m * nb; t += kBlock) {
        const int i = t / nb, c = t % nb;
        A[(size_t)(j0 + i) * n + j0 + c] = Ps[i * ld + c];
    }
}

// Apply the panel's interchanges to the columns outside [j0, j0+nb).
__global__ __launch_bounds__(kBlock) void k_lu_swap(double *__restrict__ A, int n, int j0, int nb,
                                                     const int32_t *__restrict__ piv)
{
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n - nb) return;
    const int col = t < j0 ? t : t + nb;
    for (int c = j0; c < j0 + nb; ++c) {
        const int p = piv[c];
        if (p != c) {
            const double v = A[(size_t)c * n + col];
            A[(size_t)c * n + col] = A[(size_t)p * n + col];
            A[(size_t)p * n + col] = v;
        }
    }
}

// Solve with the nb x nb diagonal block of the factor at (j0, j0) for the
// rows j0..j0+nb-1 of B (ncols columns starting at col0, leading dim ldb):
// upper = 0: unit lower triangle (forward); upper = 1: upper triangle
// (backward).  A block shorter than kNB is padded with identity rows so the
// loops are static and the column stays in registers.  Column-oriented
// updates keep up to 63 independent FMAs in flight per step.
__device__ __forceinline__ void trsm_body(const double *__restrict__ F, int n, int j0, int nb, double *B, int ldb,
                                          int col0, int ncols, int upper, int colblock)
{
    __shared__ double Ls[kNB][kNB + 1];
    for (int t = threadIdx.x; t < kNB * kNB; t += kBlock) {
        const int r = t / kNB, c = t % kNB;
        double v = (r == c) ? 1.0 : 0.0;
        if (r < nb && c < nb) v = F[(size_t)(j0 + r) * n + j0 + c];
        Ls[r][c] = v;
    }
    __syncthreads();
    const int col = col0 + colblock * kBlock + threadIdx.x;
    if (col >= col0 + ncols) return;
    double x[kNB];
#pragma unroll
    for (int r = 0; r < kNB; ++r) x[r] = (r < nb) ? B[(size_t)(j0 + r) * ldb + col] : 0.0;
    if (!upper) {
#pragma unroll
        for (int t = 0; t < kNB - 1; ++t)
#pragma unroll
            for (int r = t + 1; r < kNB; ++r) x[r] -= Ls[r][t] * x[t];
    } else {
#pragma unroll
        for (int t = kNB - 1; t >= 0; --t) {
            x[t] /= Ls[t][t];
#pragma unroll
            for (int r = 0; r < t; ++r) x[r] -= Ls[r][t] * x[t];
        }
    }
#pragma unroll
    for (int r = 0; r < kNB; ++r)
        if (r < nb) B[(size_t)(j0 + r) * ldb + col] = x[r];
}

__global__ __launch_bounds__(kBlock) void k_trsm(const double *__restrict__ F, int n, int j0, int nb, double *B,
                                                  int ldb, int col0, int ncols, int upper)
{
    trsm_body(F, n, j0, nb, B, ldb, col0, ncols, upper, blockIdx.x);
}

// ---- Gauss-Jordan inverse of an MSFE coarse matrix (symmetric positive
// definite, so the pivots are those of an unpivoted LU and stay positive):
// sweeps over 64-column panels J with D = A[J,J]:
//   A[J,J] <- D^-1,  A[J,~J] <- D^-1 A[J,~J],  A[~J,J] <- -A[~J,J] D^-1,
//   A[~J,~J] <- A[~J,~J] - A[~J,J]_old D^-1 A[J,~J]_old;
// after the last panel A holds its inverse.  The sweeps below keep only the
// lower triangle (the symmetric form further down).

// D^-1 of the nb x nb pivot block at (j0, j0) (padded to 64 x 64 with the
// identity), by one workgroup: the same sweep on entries two at a time,
// 4 x 4 entries per thread, the two pivot rows and columns through LDS (two
// buffers, one barrier per pair of pivots); written into A[J,J].
__device__ __forceinline__ void gj_pivot_wg(double *__restrict__ A, int n, int j0, int nb, int32_t *status)
{
    __shared__ double colk[2][2][kNB], rowk[2][2][kNB];
    const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
    double a[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = 4 * ti + r, j = 4 * tj + c;
            a[r][c] = (i < nb && j < nb) ? A[(size_t)(j0 + i) * n + j0 + j] : (i == j ? 1.0 : 0.0);
        }
    bool bad = false;
    // two pivots per step: with J = {k, k+1}, P = D[J,J] and Q = P^-1,
    //   D[J,J] <- Q,  D[J,~J] <- Q D[J,~J],  D[~J,J] <- -D[~J,J] Q,
    //   D[~J,~J] <- D[~J,~J] - D[~J,J] Q D[J,~J]
    // (the same sweep, two columns at a time: half the barriers, one
    // reciprocal per step)
    // the loop over the 16 tile columns stays rolled: its body (two pivot
    // pairs) is reused from the instruction cache, where the fully unrolled
    // sweep would stream every instruction once
#pragma nounroll
    for (int kg = 0; kg < kNB / 4; ++kg)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int kr = 2 * h, k = 4 * kg + kr, b = h;
        if (tj == kg)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                colk[b][0][4 * ti + r] = a[r][kr];
                colk[b][1][4 * ti + r] = a[r][kr + 1];
            }
        if (ti == kg)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                rowk[b][0][4 * tj + c] = a[kr][c];
                rowk[b][1][4 * tj + c] = a[kr + 1][c];
            }
        __syncthreads();
        const double p00 = rowk[b][0][k], p01 = rowk[b][0][k + 1], p10 = rowk[b][1][k], p11 = rowk[b][1][k + 1];
        double det = p00 * p11 - p01 * p10;
        if (!(p00 > 0.0 && p00 < 1e300 && det > 0.0 && det < 1e300)) {   // not positive definite (or not finite)
            bad = true;
            det = 1.0;
        }
        // 1/det by the hardware estimate and two Newton steps (relative error
        // near 1 ulp) instead of the correctly rounded division sequence
        double id = __builtin_amdgcn_rcp(det);
        id = id * (2.0 - det * id);
        id = id * (2.0 - det * id);
        const double q00 = p11 * id, q01 = -p01 * id, q10 = -p10 * id, q11 = p00 * id;
        double u0[4], u1[4], c0[4], c1[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double r0 = rowk[b][0][4 * tj + c], r1 = rowk[b][1][4 * tj + c];
            u0[c] = q00 * r0 + q01 * r1;
            u1[c] = q10 * r0 + q11 * r1;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            c0[r] = colk[b][0][4 * ti + r];
            c1[r] = colk[b][1][4 * ti + r];
        }
        // every entry as if off the pivot rows and columns (two FMAs), then
        // the owners of the pivot rows, columns and block overwrite theirs
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) a[r][c] -= c0[r] * u0[c] + c1[r] * u1[c];
        if (ti == kg)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                a[kr][c] = u0[c];
                a[kr + 1][c] = u1[c];
            }
        if (tj == kg)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                a[r][kr] = -(c0[r] * q00 + c1[r] * q10);
                a[r][kr + 1] = -(c0[r] * q01 + c1[r] * q11);
            }
        if (ti == kg && tj == kg) {
            a[kr][kr] = q00;
            a[kr][kr + 1] = q01;
            a[kr + 1][kr] = q10;
            a[kr + 1][kr + 1] = q11;
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = 4 * ti + r, j = 4 * tj + c;
            if (i < nb && j < nb) A[(size_t)(j0 + i) * n + j0 + j] = a[r][c];
        }
    if (bad && threadIdx.x == 0) atomicOr(status, F_SINGULAR_COARSE);
}

// Number of workgroups of a pivot step: the inverse and the copies of the
// old column block.
inline unsigned gj_pivot_wgs(int n, int nb) { return 1 + (unsigned)(((size_t)(n - nb) * nb + kBlock - 1) / kBlock); }

typedef double v4d __attribute__((ext_vector_type(4)));

// C (M x Nn, ldc) = alpha A (M x K, lda) B (K x Nn, ldb) + beta C; row-major.
// C may alias A when Nn <= 64 (each workgroup then owns whole rows of C and
// reads its rows of A before writing), or B when M <= 64 (whole columns).
// 256 threads = 4 waves as 2 x 2; each wave owns a 32 x 32 block of the
// 64 x 64 tile as 2 x 2 tiles of v_mfma_f64_16x16x4f64.  Operand lanes: A row = lane%16, k = lane/16; B col =
// lane%16, k = lane/16; result element v of a lane: row lane/16 + 4v,
// col lane%16 (checked against a host GEMM by the parity tests).
// K is staged through LDS KS = 32 columns at a time; the next stage's
// operands are loaded into registers while the matrix cores work on the
// current one (one LDS buffer, one register buffer).  With beta != 0 the
// thread's 16 elements of C are loaded with the first stage, so their
// latency hides behind the products (C is only written at the end, so an
// aliased A or B is still read before it is overwritten).
constexpr int KS = 32;
// Update launches of the symmetric sweep from kWideTilesSym tiles on take
// the lean tile at four workgroups per compute unit (a 4096^2 sweep: about
// 1950 tiles per launch, 49.6 -> 41 us per launch).
constexpr int kWideTilesSym = 1024;

//
// LEAN: no register prefetch of the next stage and C loaded only after the
// products, for 131 instead of 190 registers, so three workgroups share a
// compute unit instead of two: launches with many tiles (the rank-64 update
// of a 4096^2 sweep, 89.8 instead of 95.6 us, the same values bit for bit);
// the prefetching form stays where one round of tiles bounds the launch.
template <bool LEAN = false>
__device__ __forceinline__ void gemm_tile(double *C, int ldc, const double *A, int lda, const double *B, int ldb,
                                          int M, int Nn, int K, double alpha, double beta, int tm, int tn)
{
    __shared__ double As[64][KS + 1];
    __shared__ double Bs[KS][64 + 1];
    constexpr int PER = 64 * KS / kBlock;   // operand elements per thread and stage (8)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    v4d acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    double ra[PER], rb[PER];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int t = threadIdx.x + kBlock * i;
            const int ar = t / KS, ac = t % KS;          // A: 64 rows x KS
            const int gr = tm + ar, gc = k0 + ac;
            ra[i] = (gr < M && gc < K) ? A[(size_t)gr * lda + gc] : 0.0;
            const int br = t / 64, bc = t % 64;          // B: KS rows x 64
            const int hr = k0 + br, hc = tn + bc;
            rb[i] = (hr < K && hc < Nn) ? B[(size_t)hr * ldb + hc] : 0.0;
        }
    };
    double cv[2][2][4];
    auto load_c = [&]() {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = tm + wm + a * 16 + (lane >> 4) + 4 * v;
                    const int c = tn + wn + b * 16 + (lane & 15);
                    cv[a][b][v] = (beta != 0.0 && r < M && c < Nn) ? C[(size_t)r * ldc + c] : 0.0;
                }
    };
    if (!LEAN) {
        fetch(0);
        load_c();
    }
    for (int k0 = 0; k0 < K; k0 += KS) {
        if (LEAN) fetch(k0);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int t = threadIdx.x + kBlock * i;
            As[t / KS][t % KS] = ra[i];
            Bs[t / 64][t % 64] = rb[i];
        }
        __syncthreads();
        if (!LEAN && k0 + KS < K) fetch(k0 + KS);
#pragma unroll
        for (int kk = 0; kk < KS; kk += 4) {
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const double av = As[wm + a * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const double bv = Bs[kk + (lane >> 4)][wn + b * 16 + (lane & 15)];
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[a][b], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    if (LEAN) load_c();
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = tm + wm + a * 16 + (lane >> 4) + 4 * v;
                const int c = tn + wn + b * 16 + (lane & 15);
                if (r < M && c < Nn) {
                    const double prod = alpha * acc[a][b][v];
                    const double out = beta == 0.0 ? prod : beta * cv[a][b][v] + prod;
                    C[(size_t)r * ldc + c] = out;
                }
            }
}

// Row and column offsets of tile t of descriptor g.
__device__ __forceinline__ void tile_origin(const GemmDesc &g, int t, int &tm, int &tn)
{
    if (g.tri) {   // t = r (r + 1) / 2 + c, c <= r
        int r = (int)((__builtin_sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while (r * (r + 1) / 2 > t) --r;
        while ((r + 1) * (r + 2) / 2 <= t) ++r;
        tm = 64 * r;
        tn = 64 * (t - r * (r + 1) / 2);
    } else {
        tm = (t / g.tiles_n) * 64;
        tn = (t % g.tiles_n) * 64;
    }
}

__global__ __launch_bounds__(kBlock) void k_gemm(double *C, int ldc, const double *A, int lda, const double *B,
                                                  int ldb, int M, int Nn, int K, double alpha, double beta)
{
    gemm_tile(C, ldc, A, lda, B, ldb, M, Nn, K, alpha, beta, blockIdx.y * 64, blockIdx.x * 64);
}

// ---- batched Gauss-Jordan inverses (MSFE instances of a batch): every
// launch carries one descriptor per participating instance; a GEMM launch
// covers all tiles of all its descriptors, a pivot launch all workgroups of
// all its pivot steps.

// The pivot step whose workgroup range holds workgroup `wg` (binary search on wg0).
__device__ __forceinline__ const GjPivotDesc &pivot_desc_of(const GjPivotDesc *__restrict__ p, int np, int wg)
{
    int lo = 0, hi = np - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (p[mid].wg0 <= wg) lo = mid;
        else hi = mid - 1;
    }
    return p[lo];
}

__global__ __launch_bounds__(kBlock) void kb_gemm(const GemmDesc *__restrict__ d, int nd)
{
    // the descriptor whose tile range holds this workgroup (binary search on tile0)
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].tile0 <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const GemmDesc g = d[lo];
    int tm, tn;
    tile_origin(g, blockIdx.x - g.tile0, tm, tn);
    gemm_tile(g.C, g.ldc, g.A, g.lda, g.B, g.ldb, g.M, g.N, g.K, g.alpha, g.beta, tm, tn);
}

// ---- symmetric Gauss-Jordan sweeps (single MSFE matrices and the planes of
// the block-tridiagonal form).  The sweep keeps A[U,U] and A[S,S] symmetric
// and A[U,S] = -A[S,U]^T (S: swept columns, U: the others), so the lower
// triangle (diagonal tiles whole) determines the whole matrix and only its
// tiles are updated: half the flop and half the bytes of the full sweep.
// Per panel J (D = A[J,J], old column block Cb = A[~J,J]):
//   G = Cb D^-1;  A[J,J] <- D^-1;  A[I,J] <- -G_I (I > J);
//   A[J,K] <- -D^-1 Cb_K^T (K < J);
//   A[I,K] <- A[I,K] - s_K G_I Cb_K^T for the lower tiles I >= K outside J,
//   with s_K = +1 for K > J and -1 for K < J (A[J,K] = s_K Cb_K^T);
// where Cb_I = A[I,J] for I > J and -A[J,I]^T for I < J, both from the
// lower triangle.  After the last panel the lower triangle holds the
// inverse; k_mirror_lower copies it to the upper one.

// Workgroup 0: D^-1 (gj_pivot_wg); workgroups 1..: Cb (row stride nb) and
// its transpose CbT (nb x n, row stride n) for the rows outside J, from the
// lower triangle: rows below J from column J (nb consecutive values per
// row), rows above J from row J (consecutive along the row).
__device__ __forceinline__ void gj_pivot_sym_wg(double *__restrict__ A, int n, int j0, int nb,
                                                double *__restrict__ Cb, double *__restrict__ CbT, int32_t *status,
                                                int blk)
{
    if (blk == 0) {
        gj_pivot_wg(A, n, j0, nb, status);
        return;
    }
    const size_t t = (size_t)(blk - 1) * kBlock + threadIdx.x;
    const size_t below = (size_t)(n - j0 - nb) * nb;
    if (t < below) {
        const int i = j0 + nb + (int)(t / nb), cc = (int)(t % nb);
        const double v = A[(size_t)i * n + j0 + cc];
        Cb[(size_t)i * nb + cc] = v;
        CbT[(size_t)cc * n + i] = v;
    } else if (t < below + (size_t)j0 * nb) {
        const size_t u = t - below;
        const int cc = (int)(u / j0), i = (int)(u % j0);
        const double v = -A[(size_t)(j0 + cc) * n + i];
        Cb[(size_t)i * nb + cc] = v;
        CbT[(size_t)cc * n + i] = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_gj_pivot_sym(double *__restrict__ A, int n, int j0, int nb,
                                                          double *__restrict__ Cb, double *__restrict__ CbT,
                                                          int32_t *status)
{
    gj_pivot_sym_wg(A, n, j0, nb, Cb, CbT, status, blockIdx.x);
}

// Entry 1 of a panel of the symmetric sweep: GEMM tiles, where a descriptor
// with `pre` forms its A operand per tile in LDS as S (rows of Cb, row
// pitch lda) times pre (D^-1, row pitch ldc): the rows of G that the
// next panel's row and column need, computed by the same tile product as
// the G tiles of the same launch.
__global__ __launch_bounds__(kBlock) void k_gj_panel_sym(const GemmDesc *__restrict__ d, int nd)
{
    __shared__ double Ts[64 * 65];
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].tile0 <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const GemmDesc g = d[lo];
    int tm, tn;
    tile_origin(g, blockIdx.x - g.tile0, tm, tn);
    if (g.pre) {   // uniform over the workgroup
        const int rows = min(64, g.M - tm);
        gemm_tile(Ts, 65, g.S + (size_t)tm * g.lda, g.lda, g.pre, g.ldc, rows, g.K, g.K, 1.0, 0.0, 0, 0);
        __syncthreads();
        gemm_tile(g.C + (size_t)tm * g.ldc, g.ldc, Ts, 65, g.B, g.ldb, rows, g.N, g.K, g.alpha, g.beta, 0, tn);
    } else {
        gemm_tile(g.C, g.ldc, g.A, g.lda, g.B, g.ldb, g.M, g.N, g.K, g.alpha, g.beta, tm, tn);
    }
}

// The lower-tile update of a panel outside the next panel's row and column,
// and the next panel's pivot step (first `pw` workgroups), in one launch.
template <bool LEAN>
__device__ __forceinline__ void gj_update_pivot_sym_body(const GemmDesc *__restrict__ d, int nd, int pw, double *A,
                                                         int n, int j0, int nb, double *Cb, double *CbT,
                                                         int32_t *status)
{
    if ((int)blockIdx.x < pw) {
        gj_pivot_sym_wg(A, n, j0, nb, Cb, CbT, status, blockIdx.x);
        return;
    }
    const int tile = blockIdx.x - pw;
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].tile0 <= tile) lo = mid;
        else hi = mid - 1;
    }
    const GemmDesc g = d[lo];
    int tm, tn;
    tile_origin(g, tile - g.tile0, tm, tn);
    gemm_tile<LEAN>(g.C, g.ldc, g.A, g.lda, g.B, g.ldb, g.M, g.N, g.K, g.alpha, g.beta, tm, tn);
}
__global__ __launch_bounds__(kBlock) void k_gj_update_pivot_sym(const GemmDesc *__restrict__ d, int nd, int pw,
                                                                 double *A, int n, int j0, int nb, double *Cb,
                                                                 double *CbT, int32_t *status)
{
    gj_update_pivot_sym_body<false>(d, nd, pw, A, n, j0, nb, Cb, CbT, status);
}
// The same with the lean GEMM tile at four workgroups per compute unit.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_gj_update_pivot_sym_wide(
    const GemmDesc *__restrict__ d, int nd, int pw, double *A, int n, int j0, int nb, double *Cb, double *CbT,
    int32_t *status)
{
    gj_update_pivot_sym_body<true>(d, nd, pw, A, n, j0, nb, Cb, CbT, status);
}

// A[i][j] = A[j][i] for i < j: one workgroup per 64 x 64 tile of the
// upper triangle (tile row r < tile column c), through LDS so that reads
// and writes both run along rows.
__device__ __forceinline__ void mirror_tile(double *__restrict__ A, int n, int t)
{
    __shared__ double T[64][65];
    int c = (int)((__builtin_sqrt(8.0 * t + 1.0) - 1.0) * 0.5);   // t = c (c - 1) / 2 + r, r < c
    c += 1;
    while (c * (c - 1) / 2 > t) --c;
    while ((c + 1) * c / 2 <= t) ++c;
    const int r = t - c * (c - 1) / 2;
    const int i0 = 64 * r, j0 = 64 * c;
    // read the lower tile (rows j0.., columns i0..)
    for (int q = threadIdx.x; q < 64 * 64; q += kBlock) {
        const int a = q / 64, b = q % 64;
        if (j0 + a < n && i0 + b < n) T[a][b] = A[(size_t)(j0 + a) * n + i0 + b];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 64 * 64; q += kBlock) {
        const int a = q / 64, b = q % 64;   // upper element (i0 + a, j0 + b) = lower (j0 + b, i0 + a)
        if (i0 + a < n && j0 + b < n) A[(size_t)(i0 + a) * n + j0 + b] = T[b][a];
    }
}

__global__ __launch_bounds__(kBlock) void k_mirror_lower(double *__restrict__ A, int n)
{
    mirror_tile(A, n, blockIdx.x);
}

// ---- the symmetric sweeps of every MSFE instance of a batch, one launch
// per step for all instances that have it.

__global__ __launch_bounds__(kBlock) void kb_gj_pivot_sym(const GjPivotDesc *__restrict__ p, int np)
{
    const GjPivotDesc &q = pivot_desc_of(p, np, blockIdx.x);
    gj_pivot_sym_wg(q.A, q.n, q.j0, q.nb, q.Cb, q.CbT, q.status, blockIdx.x - q.wg0);
}

// The lower-tile update of one panel of every instance (outside the next
// panel's row and column) and the next panel's pivot steps in one launch:
// the first `pw` workgroups are the pivot steps of the next panel of every
// instance that has one, the others GEMM tiles.
template <bool LEAN>
__device__ __forceinline__ void gjb_update_pivot_body(const GjPivotDesc *__restrict__ p, int np, int pw,
                                                      const GemmDesc *__restrict__ d, int nd)
{
    if ((int)blockIdx.x < pw) {
        const GjPivotDesc &q = pivot_desc_of(p, np, blockIdx.x);
        gj_pivot_sym_wg(q.A, q.n, q.j0, q.nb, q.Cb, q.CbT, q.status, blockIdx.x - q.wg0);
        return;
    }
    const int tile = blockIdx.x - pw;
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].tile0 <= tile) lo = mid;
        else hi = mid - 1;
    }
    const GemmDesc g = d[lo];
    int tm, tn;
    tile_origin(g, tile - g.tile0, tm, tn);
    gemm_tile<LEAN>(g.C, g.ldc, g.A, g.lda, g.B, g.ldb, g.M, g.N, g.K, g.alpha, g.beta, tm, tn);
}
__global__ __launch_bounds__(kBlock) void kb_gj_update_pivot_sym(const GjPivotDesc *__restrict__ p, int np, int pw,
                                                                  const GemmDesc *__restrict__ d, int nd)
{
    gjb_update_pivot_body<false>(p, np, pw, d, nd);
}
// The same with the lean GEMM tile at four workgroups per compute unit.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void kb_gj_update_pivot_sym_wide(
    const GjPivotDesc *__restrict__ p, int np, int pw, const GemmDesc *__restrict__ d, int nd)
{
    gjb_update_pivot_body<true>(p, np, pw, d, nd);
}

// Descriptor i mirrors the matrix C (order ldc) with the tiles tile0 ..
// tile0 + T (T - 1) / 2 - 1 of the launch (T = tiles_n).
__global__ __launch_bounds__(kBlock) void kb_mirror_lower(const GemmDesc *__restrict__ d, int nd)
{
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].tile0 <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    mirror_tile(d[lo].C, d[lo].ldc, blockIdx.x - d[lo].tile0);
}

// B = P I for the row interchanges of the factorisation (one thread builds
// the permutation, then every thread fills a row).
__global__ __launch_bounds__(kBlock) void k_perm_identity(const int32_t *__restrict__ piv, int n,
                                                           int32_t *__restrict__ perm, double *__restrict__ B)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int i = 0; i < n; ++i) perm[i] = i;
        for (int c = 0; c < n; ++c) {
            const int p = piv[c];
            const int t = perm[c];
            perm[c] = perm[p];
            perm[p] = t;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_perm_fill(const int32_t *__restrict__ perm, int n, double *__restrict__ B)
{
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (size_t)n * n) return;
    const int i = (int)(t / n), j = (int)(t % n);
    B[t] = (perm[i] == j) ? 1.0 : 0.0;
}

__global__ __launch_bounds__(kBlock) void k_copy(const double *__restrict__ a, double *__restrict__ b, size_t n)
{
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < n) b[t] = a[t];
}

// (R r)_k from the owner-box slot partials of the restriction: MSFE adds,
// in a fixed order, slot (dx + 2 dy + 4 dz) of the box k - (dx, dy, dz) for
// the boxes that exist; MSFV takes slot 0 of box k.
__device__ __forceinline__ double node_sum(const GridDev &g, const double *__restrict__ slots, int fe, int k)
{
    if (!fe) return slots[(size_t)k * 8];
    const int ka = k % g.nb[0], kb = (k / g.nb[0]) % g.nb[1], kc = k / (g.nb[0] * g.nb[1]);
    // the eight loads from clamped addresses, outside any branch, so that
    // they are in flight together; slots outside the grid add zero
    double v[8];
    bool ok[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int a = ka - (q & 1), b = kb - ((q >> 1) & 1), c = kc - (q >> 2);
        ok[q] = a >= 0 && b >= 0 && c >= 0;
        v[q] = slots[(size_t)node_index(g, max(a, 0), max(b, 0), max(c, 0)) * 8 + q];
    }
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += ok[q] ? v[q] : 0.0;
    return s;
}

__global__ __launch_bounds__(kBlock) void k_node_sum(GridDev g, const double *__restrict__ slots, int fe,
                                                      double *__restrict__ rc, const int32_t *done)
{
    if (done && *done) return;
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= g.Nc) return;
    rc[k] = node_sum(g, slots, fe, k);
}


// Dot product of the row mr (n entries) with x by one wave: 16-byte loads,
// four in flight per lane, four independent sums when n is a multiple of 512
// (mr and x then 16-byte aligned), else one entry per lane and step.
__device__ __forceinline__ double row_dot(const double *__restrict__ mr, const double *__restrict__ x, int n,
                                          int lane)
{
    double s = 0.0;
    if (n % 512 == 0) {
        typedef double d2 __attribute__((ext_vector_type(2)));
        const d2 *m2 = (const d2 *)mr, *x2 = (const d2 *)x;
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        for (int c = lane; c < n / 2; c += 256) {
            d2 mv[4], xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                mv[u] = m2[c + 64 * u];
                xv[u] = x2[c + 64 * u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] += mv[u].x * xv[u].x + mv[u].y * xv[u].y;
        }
        s = (a[0] + a[1]) + (a[2] + a[3]);
    } else {
        for (int c = lane; c < n; c += 64) s += mr[c] * x[c];
    }
    return wave_sum(s);
}

// y = M x, one wave per row (fixed lane partition and shuffle tree).  With
// `slots` set (n <= kGemvLds), x = R r is first assembled in LDS from the
// restriction's slot partials.
//
// With `partial` set, one extra workgroup (the last) runs the stopping test
// of the iteration on the residual partials instead (stop_test), in parallel
// with the rows.  The test may set the done flag while the row workgroups
// start: a row workgroup that sees it skips its row, which is then unused.
__global__ __launch_bounds__(kBlock) void k_gemv(const double *__restrict__ M, int n, const double *__restrict__ x,
                                                  GridDev g, const double *__restrict__ slots, int fe,
                                                  double *__restrict__ y, const int32_t *done,
                                                  const double *__restrict__ partial, int nparts, int32_t *ictl,
                                                  double *scal, double rtol2, int maxit)
{
    static_assert(kBlock == kStopThreads, "one workgroup shape for the rows and the stopping test");
    __shared__ double xs[kGemvLds];
    if (done && *done) return;
    if (partial && blockIdx.x == gridDim.x - 1) {
        stop_test(partial, nparts, ictl, scal, rtol2, maxit, xs);
        return;
    }
    const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const double *mr = M + (size_t)(row < n ? row : 0) * n;
    if (slots) {
        // R r formed in LDS: the row's entries are loaded first, so that
        // their latency overlaps the node sums (n <= kGemvLds)
        constexpr int Q = kGemvLds / 64;
        double mv[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) mv[q] = lane + 64 * q < n ? mr[lane + 64 * q] : 0.0;
        for (int k = threadIdx.x; k < n; k += kBlock) xs[k] = node_sum(g, slots, fe, k);
        __syncthreads();
        if (row >= n) return;
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (lane + 64 * q < n) s += mv[q] * xs[lane + 64 * q];
        s = wave_sum(s);
        if (lane == 0) y[row] = s;
        return;
    }
    if (row >= n) return;
    const double s = row_dot(mr, x, n, lane);
    if (lane == 0) y[row] = s;
}

// y = M x for a symmetric M (the dense MSFE inverse) reading only its lower
// triangle: one workgroup per 64 x 64 tile (I, J), J <= I (a lane reads a
// 4 x 4 sub-block; row and column sums by lane exchanges, so the workgroup
// needs 3 KB of LDS), forms x_J and x_I
// = (R r) from the restriction's slot partials, reads the tile once and
// writes (M_IJ x_J) to part[I][J] and, below the diagonal, (M_IJ^T x_I) to
// part[J][I] (64 values each); k_gemv_sym_reduce sums part[I][0..T) in a
// fixed order.  The diagonal tiles also store x_I in rc.  Half the bytes of
// the row-wise product.  With `partial` set one extra workgroup (the last)
// runs the iteration's stopping test.  TM: the stored entries, FP64 or
// (mixed-precision solves) the inverse rounded to FP32; sums in FP64.
template <class TM>
__global__ __launch_bounds__(kBlock) void k_gemv_sym(const TM *__restrict__ M, int n, GridDev g,
                                                      const double *__restrict__ slots, int fe,
                                                      double *__restrict__ rc, double *__restrict__ part,
                                                      const int32_t *done, const double *__restrict__ partial,
                                                      int nparts, int32_t *ictl, double *scal, double rtol2,
                                                      int maxit)
{
    static_assert(kBlock == 256 && kBlock == kStopThreads, "four waves per tile; one workgroup shape");
    __shared__ double xs[2][64];
    __shared__ double red[4][64];
    if (done && *done) return;
    if (partial && blockIdx.x == gridDim.x - 1) {
        stop_test(partial, nparts, ictl, scal, rtol2, maxit, &red[0][0]);
        return;
    }
    const int t = blockIdx.x;   // t = I (I + 1) / 2 + J
    int I = (int)((__builtin_sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > t) --I;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int J = t - I * (I + 1) / 2, T = (n + 63) / 64;
    const int i0 = 64 * I, j0 = 64 * J;
    // wave w takes tile rows 16 w .. 16 w + 15; lane: 4 x 4 sub-block at rows
    // 16 w + 4 rq + k (k < 4), columns 4 cq + c (c < 4), rq = lane / 16,
    // cq = lane % 16, so each row of the wave is read by 16 lanes, 512
    // contiguous bytes.  The tile's loads first.
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, rq = lane >> 4, cq = lane & 15;
    const int rbase = 16 * w + 4 * rq, cbase = 4 * cq;
    double a[4][4];
    if (i0 + 64 <= n && j0 + 64 <= n && n % (16 / (int)sizeof(TM)) == 0) {   // whole tile, 16-byte aligned rows
        if constexpr (sizeof(TM) == 8) {
            typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const d2 *row = (const d2 *)(M + (size_t)(i0 + rbase + k) * n + j0 + cbase);
                const d2 v0 = row[0], v1 = row[1];
                a[k][0] = v0.x;
                a[k][1] = v0.y;
                a[k][2] = v1.x;
                a[k][3] = v1.y;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float4 v = *(const float4 *)(M + (size_t)(i0 + rbase + k) * n + j0 + cbase);
                a[k][0] = v.x;
                a[k][1] = v.y;
                a[k][2] = v.z;
                a[k][3] = v.w;
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int r = i0 + rbase + k, cc = j0 + cbase + c;
                a[k][c] = r < n && cc < n ? (double)M[(size_t)r * n + cc] : 0.0;
            }
    }
    if (tid < 128) {
        const int h = tid >> 6, k = (h ? i0 : j0) + (tid & 63);
        xs[h][tid & 63] = k < n ? node_sum(g, slots, fe, k) : 0.0;
    }
    __syncthreads();
    // row products: the lane's 4 rows over its 4 columns, then summed over the
    // 16 lanes of the row quad (xor over the lane's low four bits)
    double ur[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) s += a[k][c] * xs[0][cbase + c];
        ur[k] = s;
    }
#pragma unroll
    for (int m = 1; m < 16; m <<= 1)
#pragma unroll
        for (int k = 0; k < 4; ++k) ur[k] += __shfl_xor(ur[k], m);
    if (cq == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i0 + rbase + k < n) part[((size_t)I * T + J) * 64 + rbase + k] = ur[k];
    if (I == J) {
        if (tid < 64 && i0 + tid < n) rc[i0 + tid] = xs[1][tid];
        return;   // uniform over the workgroup
    }
    // transposed product: the lane's 4 columns over its 4 rows, summed over
    // the wave's four row quads (xor 16, 32), then over the four waves in LDS
    double uc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) s += a[k][c] * xs[1][rbase + k];
        uc[c] = s;
    }
#pragma unroll
    for (int m = 16; m < 64; m <<= 1)
#pragma unroll
        for (int c = 0; c < 4; ++c) uc[c] += __shfl_xor(uc[c], m);
    if (rq == 0)
#pragma unroll
        for (int c = 0; c < 4; ++c) red[w][cbase + c] = uc[c];
    __syncthreads();
    if (tid < 64 && j0 + tid < n)
        part[((size_t)J * T + I) * 64 + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
}

// M32 = M rounded to FP32 on the 64 x 64 tiles (I, J), J <= I, that
// k_gemv_sym reads (one workgroup per tile, t = I (I + 1) / 2 + J).
__global__ __launch_bounds__(kBlock) void k_round_lower(const double *__restrict__ M, float *__restrict__ M32, int n)
{
    const int t = blockIdx.x;
    int I = (int)((__builtin_sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > t) --I;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int J = t - I * (I + 1) / 2;
    for (int q = threadIdx.x; q < 64 * 64; q += kBlock) {
        const int r = 64 * I + q / 64, cc = 64 * J + q % 64;
        if (r < n && cc < n) M32[(size_t)r * n + cc] = (float)M[(size_t)r * n + cc];
    }
}

// y[i] = sum over J of part[I][J][i mod 64] (I = i / 64), J ascending.
__global__ __launch_bounds__(kBlock) void k_gemv_sym_reduce(const double *__restrict__ part, int n,
                                                             double *__restrict__ y, const int32_t *done)
{
    if (done && *done) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int T = (n + 63) / 64, I = i / 64;
    const double *p = part + (size_t)I * T * 64 + (i % 64);
    // eight independent sums (J mod 8), combined in a fixed order
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int J = 0;
    for (; J + 8 <= T; J += 8)
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] += p[(size_t)(J + k) * 64];
    for (int k = 0; J + k < T; ++k) acc[k] += p[(size_t)(J + k) * 64];
    y[i] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// Two independent products y = alpha M x + beta y with m x m matrices (row
// pitch m) in one launch, for the two chains of the block-tridiagonal
// substitutions, one wave per row: rows [0, m) of the launch are the first
// product's, [m, 2m) the second's (rows = m runs the first alone).
struct GemvJob {
    const double *M, *x;
    double *y;
    double alpha, beta;
};
__global__ __launch_bounds__(kBlock) void k_gemv_pair(GemvJob j0, GemvJob j1, int m, int rows, const int32_t *done)
{
    if (done && *done) return;
    const int R = (int)blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (R >= rows) return;
    const bool second = R >= m;
    const GemvJob j = second ? j1 : j0;
    const int row = R - (second ? m : 0);
    const double s = row_dot(j.M + (size_t)row * m, j.x, m, lane);
    if (lane == 0) j.y[row] = j.beta == 0.0 ? j.alpha * s : j.beta * j.y[row] + j.alpha * s;
}

// y_k = E_k x_k for every plane k at once (E: the planes' m x m blocks one
// after another, so row R of the launch is row R of E; x, y: m per plane),
// one wave per row.
__global__ __launch_bounds__(kBlock) void k_gemv_planes(const double *__restrict__ E, int m, size_t rows,
                                                         const double *__restrict__ x, double *__restrict__ y,
                                                         const int32_t *done)
{
    if (done && *done) return;
    const size_t R = (size_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (R >= rows) return;
    const double s = row_dot(E + R * m, x + (R / m) * m, m, threadIdx.x & 63);
    if ((threadIdx.x & 63) == 0) y[R] = s;
}

// dst (rows x cols, ldd) = src (lds)
__global__ __launch_bounds__(kBlock) void k_copy2d(const double *__restrict__ src, int lds, double *__restrict__ dst,
                                                    int ldd, int rows, int cols)
{
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (size_t)rows * cols) return;
    const int r = (int)(t / cols), c = (int)(t % cols);
    dst[(size_t)r * ldd + c] = src[(size_t)r * lds + c];
}

// ---- products with the off-diagonal plane blocks of the block-tridiagonal
// coarse operator.  Node (a, b) of one coarse z-plane couples only with the
// nodes (a + da, b + db), |da|, |db| <= 1, of the adjacent planes (the
// 27-point coarse stencil; every other entry of A_c is exactly zero), so a
// product with such a block sums 9 terms, in the fixed order q = 3 (db + 1)
// + (da + 1), instead of m.

// Plane-neighbour q of node r (nbx nodes per row of the plane), or -1.
__device__ __forceinline__ int plane_nb(int r, int q, int nbx, int nby)
{
    const int a = r % nbx + (q % 3) - 1, b = r / nbx + (q / 3) - 1;
    return (a >= 0 && a < nbx && b >= 0 && b < nby) ? a + nbx * b : -1;
}

// F (m x m) = L E: L = the block of A_c at (plane k, plane k - 1) (leading
// dimension ldl), E (m x m).  One workgroup per (row r, 256 columns).
__global__ __launch_bounds__(kBlock) void k_plane_left(double *__restrict__ F, const double *__restrict__ L, int ldl,
                                                        const double *__restrict__ E, int m, int nbx, int nby)
{
    const int r = blockIdx.y;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= m) return;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int c = plane_nb(r, q, nbx, nby);
        if (c >= 0) s += L[(size_t)r * ldl + c] * E[(size_t)c * m + j];
    }
    F[(size_t)r * m + j] = s;
}

// Uc (m x 9): the nonzeros of each column j of U (the block of A_c at
// (plane k - 1, plane k), leading dimension ldu), Uc[j][q] = U[c_q(j)][j].
__global__ __launch_bounds__(kBlock) void k_plane_cols(double *__restrict__ Uc, const double *__restrict__ U, int ldu,
                                                        int m, int nbx, int nby)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= 9 * m) return;
    const int j = t / 9, q = t % 9;
    const int c = plane_nb(j, q, nbx, nby);
    Uc[t] = c >= 0 ? U[(size_t)c * ldu + j] : 0.0;
}

// Out (m x m) = X U (sub = 0) or Out -= X U (sub = 1), X (m x m), U given
// by its column nonzeros Uc.  One thread per element.
__global__ __launch_bounds__(kBlock) void k_plane_right(double *__restrict__ Out, const double *__restrict__ X,
                                                         const double *__restrict__ Uc, int m, int nbx, int nby,
                                                         int sub)
{
    const int r = blockIdx.y;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= m) return;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int c = plane_nb(j, q, nbx, nby);
        if (c >= 0) s += X[(size_t)r * m + c] * Uc[(size_t)j * 9 + q];
    }
    double *o = Out + (size_t)r * m + j;
    *o = sub ? *o - s : s;
}

// Batched coarse solve: rc = R r from the slot partials (work item = block
// of kBlock coarse nodes), then xc = Ainv rc (work item = kBlock/64 rows).
__global__ __launch_bounds__(kBlock) void kb_node_sum(const InstDev *__restrict__ inst,
                                                       const WorkItem *__restrict__ work, const int32_t *nwork)
{
    CAMS_FOR_ITEMS(t, nwork)
    {
        const WorkItem w = work[t];
        const InstDev &d = inst[w.inst];
        if (d.a.ictl[C_DONE]) continue;
        const int k = w.blk * kBlock + threadIdx.x;
        if (k < d.g.Nc) d.a.rc[k] = node_sum(d.g, d.a.slots, d.fe, k);
    }
}

__global__ __launch_bounds__(kBlock) void kb_gemv(const InstDev *__restrict__ inst, const WorkItem *__restrict__ work,
                                                   const int32_t *nwork)
{
    CAMS_FOR_ITEMS(t, nwork)
    {
        const WorkItem w = work[t];
        const InstDev &d = inst[w.inst];
        if (d.a.ictl[C_DONE]) continue;
        const int n = d.g.Nc;
        const int row = w.blk * (kBlock / 64) + (threadIdx.x >> 6);
        const int lane = threadIdx.x & 63;
        if (row >= n) continue;   // whole waves: no workgroup barrier follows
        const double *mr = d.a.Ainv + (size_t)row * n;
        const double *x = d.a.rc;
        double s = 0.0;
        for (int c = lane; c < n; c += 64) s += mr[c] * x[c];
        s = wave_sum(s);
        if (lane == 0) d.a.xc[row] = s;
    }
}

inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

void gemm(cams_ctx *c, double *C, int ldc, const double *A, int lda, const double *B, int ldb, int M, int Nn, int K,
          double alpha, double beta)
{
    if (M <= 0 || Nn <= 0 || K <= 0) return;
    dim3 grid(cdiv(Nn, 64), cdiv(M, 64));
    k_gemm<<<grid, kBlock, 0, c->stream>>>(C, ldc, A, lda, B, ldb, M, Nn, K, alpha, beta);
}

// C -= A B
void gemm_sub(cams_ctx *c, double *C, int ldc, const double *A, int lda, const double *B, int ldb, int M, int Nn,
              int K)
{
    gemm(c, C, ldc, A, lda, B, ldb, M, Nn, K, -1.0, 1.0);
}


}  // namespace

void launch_zero_coarse(cams_ctx *c)
{
    const int n = c->g.Nc;
    if (!c->ac_zeroed) {   // entries outside the 27-point pattern stay zero from now on
        k_zero<<<cdiv((size_t)n * n, kBlock), kBlock, 0, c->stream>>>(c->a.Ac, (size_t)n * n);
        c->ac_zeroed = true;
    }
}

void launch_coarse_change(cams_ctx *c, bool snap)
{
    const int n = 27 * c->g.Nc, nb = (int)cdiv(n, kBlock);
    k_coarse_change<<<nb, kBlock, 0, c->stream>>>(c->g, c->a.Ac, c->a.Acs, snap ? 1 : 0, c->a.partial);
    if (!snap) k_max_reduce<<<1, kBlock, 0, c->stream>>>(c->a.partial, nb, c->a.scal + S_CCHG);
}

void launch_coarse_operator(cams_ctx *c)
{
    const int n = c->g.Nc;
    if (c->opt.restriction != CAMS_R_FE) {
        k_coarse_row<<<n, kBlock, 0, c->stream>>>(c->g, c->a.W, c->a.diag, c->a.dmask, c->a.P, 0, c->a.Ac);
        return;
    }
    launch_zero_coarse(c);
    k_coarse_box<<<n, kOpThreads, 0, c->stream>>>(c->g, c->a.W, c->a.diag, c->a.dmask, c->a.P, c->a.boxp);
    k_coarse_nodes<<<cdiv((size_t)27 * n, kBlock), kBlock, 0, c->stream>>>(c->g, c->a.boxp, c->a.Ac);
}

// Descriptors of the symmetric sweep of A (n x n): three launch entries per
// panel p, each (offset, count, tiles) in L:
//   1. G = Cb D^-1 and the panel: A[I,J] = -Cb_I D^-1 (I > J),
//      A[J,K] = -D^-1 CbT_K (K < J); in the same launch the lower tiles of
//      the next panel's row (K < J) and column (I >= J2), whose tiles form
//      their rows of G themselves (pre = D^-1, S = Cb: k_gj_panel_sym);
//   2. empty;
//   3. the other lower tiles outside J (launched with the next pivot step).
// Cb[p & 1] / CbT[p & 1] hold panel p's old column block (row stride nb) and
// its transpose (row stride n); G (row stride nb) is rewritten per panel.
static void gj_plan_sym(double *A, int n, double *const Cb[2], double *const CbT[2], double *G,
                        std::vector<GemmDesc> &d, std::vector<int> &L)
{
    std::vector<GemmDesc> v;
    auto add = [&](double *C, int ldc, const double *Aop, int lda, const double *B, int ldb, int M, int N, int K,
                   double al, double be, int tri) {
        if (M <= 0 || N <= 0 || K <= 0) return;
        GemmDesc g{};
        g.C = C;
        g.A = Aop;
        g.B = B;
        g.ldc = ldc;
        g.lda = lda;
        g.ldb = ldb;
        g.M = M;
        g.N = N;
        g.K = K;
        g.alpha = al;
        g.beta = be;
        g.tiles_n = (int)cdiv(N, 64);
        g.tri = tri;
        v.push_back(g);
    };
    auto flush = [&]() {
        int tiles = 0;
        for (GemmDesc &g : v) {
            g.tile0 = tiles;
            tiles += g.tri ? g.tiles_n * (g.tiles_n + 1) / 2 : g.tiles_n * (int)cdiv(g.M, 64);
        }
        L.push_back((int)d.size());
        L.push_back((int)v.size());
        L.push_back(tiles);
        d.insert(d.end(), v.begin(), v.end());
        v.clear();
    };
    for (int p = 0, j0 = 0; j0 < n; ++p, j0 += kNB) {
        const int nb = std::min(kNB, n - j0), j1 = j0 + nb, rest = n - j1;
        const int nb1 = std::min(kNB, rest), j2 = j1 + nb1;   // next panel (width 0 after the last)
        double *const cb = Cb[p & 1], *const cbt = CbT[p & 1];
        const double *Dq = A + (size_t)j0 * n + j0;
        // 1. G rows outside J, then the two parts of the panel
        add(G, nb, cb, nb, Dq, n, j0, nb, nb, 1.0, 0.0, 0);
        add(G + (size_t)j1 * nb, nb, cb + (size_t)j1 * nb, nb, Dq, n, rest, nb, nb, 1.0, 0.0, 0);
        add(A + (size_t)j1 * n + j0, n, cb + (size_t)j1 * nb, nb, Dq, n, rest, nb, nb, -1.0, 0.0, 0);
        add(A + (size_t)j0 * n, n, Dq, n, cbt, n, nb, j0, nb, -1.0, 0.0, 0);
        // next panel's row (K < J: s_K = -1) and column (rows from J2 on: s_K = +1),
        // the A operand G_I formed per tile as Cb_I D^-1
        const size_t before = v.size();
        add(A + (size_t)j1 * n, n, nullptr, nb, cbt, n, nb1, j0, nb, 1.0, 1.0, 0);
        add(A + (size_t)j1 * n + j1, n, nullptr, nb, cbt + j1, n, rest, nb1, nb, -1.0, 1.0, 0);
        for (size_t i = before; i < v.size(); ++i) {
            v[i].pre = Dq;
            v[i].S = cb + (size_t)j1 * nb;
        }
        flush();
        flush();   // the second entry stays empty
        // 3. the rest: K < J (triangle above J, rectangle below the next row), K > J2 (triangle)
        add(A, n, G, nb, cbt, n, j0, j0, nb, 1.0, 1.0, 1);
        add(A + (size_t)j2 * n, n, G + (size_t)j2 * nb, nb, cbt, n, n - j2, j0, nb, 1.0, 1.0, 0);
        add(A + (size_t)j2 * n + j2, n, G + (size_t)j2 * nb, nb, cbt + j2, n, n - j2, n - j2, nb, -1.0, 1.0, 1);
        flush();
    }
}

// Buffers of the symmetric sweeps of chain `ch` (the block-tridiagonal form
// runs two elimination chains at once; everything else uses chain 0): the
// two old column blocks (m x kNB each), their transposes (kNB x m each) and
// G (m x kNB).
struct GjBufs {
    double *Cb[2], *CbT[2], *G;
};
static GjBufs gj_bufs(const cams_ctx *c, int m, int ch)
{
    const size_t blk = (size_t)m * kNB;
    double *const base = c->a.gjcb + (size_t)ch * (5 * blk + 64 * 64);
    return GjBufs{{base, base + blk}, {base + 2 * blk, base + 3 * blk}, base + 4 * blk};
}

// The descriptors of every matrix the factorisation inverts, uploaded once
// per workspace (the matrices live at fixed places in it); matrix i uses the
// buffers of chain chains[i].
static void gj_prepare(cams_ctx *c, const std::vector<double *> &mats, const std::vector<int> &chains, int m)
{
    if (c->gj_ready) return;
    std::vector<GemmDesc> d;
    c->gj_launch.clear();
    for (size_t i = 0; i < mats.size(); ++i) {
        const GjBufs b = gj_bufs(c, m, chains[i]);
        gj_plan_sym(mats[i], m, b.Cb, b.CbT, b.G, d, c->gj_launch);
    }
    if (!d.empty())
        CAMS_HIP(hipMemcpyAsync(c->a.gjd, d.data(), d.size() * sizeof(GemmDesc), hipMemcpyHostToDevice, c->stream));
    CAMS_HIP(hipStreamSynchronize(c->stream));   // d is a local buffer
    c->gj_ready = true;
}

// In-place inverse of matrix `mat` (the mat-th of gj_prepare's list), m x m,
// by the symmetric sweep: the first pivot step, then per panel the panel
// products with the next panel's row and column (one launch), and the rest
// of the update together with the next pivot step; finally the lower
// triangle is copied to the upper one.  Enqueued on stream st with the buffers of chain ch (as
// given to gj_prepare for this matrix).
static void inverse_gj(cams_ctx *c, double *A, int m, int mat, int ch, hipStream_t st)
{
    const int panels = (m + kNB - 1) / kNB;
    const GemmDesc *dd = (const GemmDesc *)c->a.gjd;
    const GjBufs b = gj_bufs(c, m, ch);
    const int nb0 = std::min(kNB, m);
    k_gj_pivot_sym<<<gj_pivot_wgs(m, nb0), kBlock, 0, st>>>(A, m, 0, nb0, b.Cb[0], b.CbT[0], c->a.status);
    for (int p = 0; p < panels; ++p) {
        const int *e = &c->gj_launch[3 * 3 * (mat * panels + p)];
        if (e[1] > 0) k_gj_panel_sym<<<e[2], kBlock, 0, st>>>(dd + e[0], e[1]);
        e += 6;   // the second entry is empty
        const int j1 = (p + 1) * kNB;
        if (j1 < m) {
            const int nb1 = std::min(kNB, m - j1), q = (p + 1) & 1;
            const unsigned pw = gj_pivot_wgs(m, nb1);
            if (e[2] >= kWideTilesSym)
                k_gj_update_pivot_sym_wide<<<pw + e[2], kBlock, 0, st>>>(dd + e[0], e[1], (int)pw, A, m, j1, nb1,
                                                                         b.Cb[q], b.CbT[q], c->a.status);
            else
                k_gj_update_pivot_sym<<<pw + e[2], kBlock, 0, st>>>(dd + e[0], e[1], (int)pw, A, m, j1, nb1,
                                                                    b.Cb[q], b.CbT[q], c->a.status);
        } else if (e[1] > 0) {
            kb_gemm<<<e[2], kBlock, 0, st>>>(dd + e[0], e[1]);
        }
    }
    if (panels > 1) k_mirror_lower<<<panels * (panels - 1) / 2, kBlock, 0, st>>>(A, m);
}

// ---- batched MSFE factorisation: the Gauss-Jordan sweeps of every FE
// instance of a batch, one launch per step for all instances (the same
// steps as inverse_gj, in place in each instance's Ainv).

// Saved column blocks of an instance's dense sweep: its own buffer, or for
// an instance that factorises by planes when alone (its buffer is sized for
// one plane) the working matrix, which the dense sweep does not use.
static GjBufs batch_gj_bufs(const cams_ctx *c)
{
    const size_t blk = (size_t)c->g.Nc * kNB;
    double *base = c->blocktri ? c->a.work : c->a.gjcb;
    return GjBufs{{base, base + blk}, {base + 2 * blk, base + 3 * blk}, base + 4 * blk};
}

// Per instance: A_c copied into Ainv, which the sweeps invert in place.
void launch_coarse_factor_prepare(cams_ctx *c)
{
    c->ainv32_ok = false;   // the batched sweeps rewrite Ainv without rounding it
    const size_t nn = (size_t)c->g.Nc * c->g.Nc;
    k_copy<<<cdiv(nn, kBlock), kBlock, 0, c->stream>>>(c->a.Ac, c->a.Ainv, nn);
}

void plan_batch_gj(const std::vector<cams_ctx *> &fe, BatchGjPlan &plan)
{
    plan = BatchGjPlan();
    const int m = (int)fe.size();
    std::vector<std::vector<GemmDesc>> d(m);
    std::vector<std::vector<int>> L(m);
    int maxP = 0;
    for (int i = 0; i < m; ++i) {
        const cams_ctx *c = fe[i];
        const GjBufs bf = batch_gj_bufs(c);
        gj_plan_sym(c->a.Ainv, c->g.Nc, bf.Cb, bf.CbT, bf.G, d[i], L[i]);
        maxP = std::max(maxP, (c->g.Nc + kNB - 1) / kNB);
    }
    // pivot steps of panel p of every instance that has it
    auto pivots = [&](int p, int &count, int &wgs) -> size_t {
        const size_t off = plan.piv.size();
        wgs = 0;
        for (int i = 0; i < m; ++i) {
            const cams_ctx *c = fe[i];
            const int n = c->g.Nc, j0 = p * kNB;
            if (j0 >= n) continue;
            const int nb = std::min(kNB, n - j0);
            const GjBufs bf = batch_gj_bufs(c);
            plan.piv.push_back(GjPivotDesc{c->a.Ainv, bf.Cb[p & 1], bf.CbT[p & 1], c->a.status, n, j0, nb, wgs});
            wgs += (int)gj_pivot_wgs(n, nb);
        }
        count = (int)(plan.piv.size() - off);
        return off;
    };
    // launch entry h (0: panel, 2: update) of panel p of every instance, tiles renumbered
    auto gemms = [&](int p, int h, int &count, int &tiles) -> size_t {
        const size_t off = plan.gemms.size();
        tiles = 0;
        for (int i = 0; i < m; ++i) {
            const int panels = (fe[i]->g.Nc + kNB - 1) / kNB;
            if (p >= panels) continue;
            const int *e = &L[i][3 * (3 * p + h)];
            for (int k = 0; k < e[1]; ++k) {
                GemmDesc g = d[i][e[0] + k];
                g.tile0 += tiles;
                plan.gemms.push_back(g);
            }
            tiles += e[2];
        }
        count = (int)(plan.gemms.size() - off);
        return off;
    };
    BatchGjPlan::Launch first{BatchGjPlan::PIVOT, 0, 0, 0, 0, 0, 0};
    first.poff = pivots(0, first.pcount, first.pw);
    plan.launches.push_back(first);
    for (int p = 0; p < maxP; ++p) {
        BatchGjPlan::Launch g{BatchGjPlan::PANEL, 0, 0, 0, 0, 0, 0};
        g.goff = gemms(p, 0, g.gcount, g.tiles);
        if (g.gcount > 0) plan.launches.push_back(g);
        BatchGjPlan::Launch u{BatchGjPlan::UPDATE_PIVOT, 0, 0, 0, 0, 0, 0};
        u.poff = pivots(p + 1, u.pcount, u.pw);
        u.goff = gemms(p, 2, u.gcount, u.tiles);
        if (u.pcount + u.gcount > 0) plan.launches.push_back(u);
    }
    // the lower triangles to the upper ones, every instance in one launch
    BatchGjPlan::Launch mr{BatchGjPlan::MIRROR, 0, 0, 0, 0, 0, 0};
    mr.goff = plan.gemms.size();
    for (int i = 0; i < m; ++i) {
        const int n = fe[i]->g.Nc, T = (n + 63) / 64;
        if (T < 2) continue;
        GemmDesc g{};
        g.C = fe[i]->a.Ainv;
        g.ldc = n;
        g.tiles_n = T;
        g.tile0 = mr.tiles;
        plan.gemms.push_back(g);
        mr.tiles += T * (T - 1) / 2;
    }
    mr.gcount = (int)(plan.gemms.size() - mr.goff);
    if (mr.gcount > 0) plan.launches.push_back(mr);
}

void launch_batch_gj(const BatchGjPlan &plan, const GjPivotDesc *piv, const GemmDesc *gemms, hipStream_t st)
{
    for (const BatchGjPlan::Launch &L : plan.launches) {
        if (L.kind == BatchGjPlan::PIVOT) {
            if (L.pcount > 0) kb_gj_pivot_sym<<<L.pw, kBlock, 0, st>>>(piv + L.poff, L.pcount);
        } else if (L.kind == BatchGjPlan::PANEL) {
            k_gj_panel_sym<<<L.tiles, kBlock, 0, st>>>(gemms + L.goff, L.gcount);
        } else if (L.kind == BatchGjPlan::MIRROR) {
            kb_mirror_lower<<<L.tiles, kBlock, 0, st>>>(gemms + L.goff, L.gcount);
        } else if (L.pcount > 0) {
            if (L.tiles >= kWideTilesSym)
                kb_gj_update_pivot_sym_wide<<<L.pw + L.tiles, kBlock, 0, st>>>(piv + L.poff, L.pcount, L.pw,
                                                                               gemms + L.goff, L.gcount);
            else
                kb_gj_update_pivot_sym<<<L.pw + L.tiles, kBlock, 0, st>>>(piv + L.poff, L.pcount, L.pw,
                                                                          gemms + L.goff, L.gcount);
        } else if (L.gcount > 0) {
            kb_gemm<<<L.tiles, kBlock, 0, st>>>(gemms + L.goff, L.gcount);
        }
    }
}

// Blocks of the block-tridiagonal form (coarse nodes ordered plane by plane
// in z, m = nb_x nb_y nodes per plane, Z planes, L_k / U_k the blocks that
// couple plane k with planes k - 1 / k + 1), eliminated from both ends
// towards the twist plane t = (Z - 1) / 2, so the two chains of dense
// inversions run at the same time:
//   top, k < t:     S_0 = D_0, S_k = D_k - F_k U_{k-1},  F_k = L_k E_{k-1},
//                   G_k = E_k U_k;
//   bottom, k > t:  S_{Z-1} = D_{Z-1}, S_k = D_k - H_k L_{k+1},
//                   H_k = U_k E_{k+1},  K_k = E_k L_k;
//   twist:          S_t = D_t - F_t U_{t-1} - H_t L_{t+1};
// E_k = S_k^-1 for every plane.  Stored in Ainv as E (Z m^2), then F_k at
// slot k (k = 1..t) and H_k at slot k + 1 (k = t..Z-2), then G_k at slot k
// (k < t) and K_k at slot k (k > t).
static void blocktri_parts(const cams_ctx *c, double *&E, double *&Fk, double *&G, int &m, int &Z)
{
    m = c->g.nb[0] * c->g.nb[1];
    Z = c->g.nb[2];
    const size_t mm = (size_t)m * m;
    E = c->a.Ainv;
    Fk = E + Z * mm;
    G = Fk + Z * mm;
}

inline int twist_plane(int Z) { return (Z - 1) / 2; }

// A_c of an MSFE problem couples only nodes of adjacent z-planes (a basis
// function vanishes on the vertex planes next to its own), so the coarse
// operator is block tridiagonal by planes.  Factorisation by block
// elimination from both ends: Z dense m x m inversions on matrix cores
// instead of one Nc x Nc inversion (Nc = Z m), at most Z - t of them in
// sequence (the bottom chain runs on the context's second stream); the
// products with the off-diagonal plane blocks use their 9-point sparsity.
static void factor_blocktri(cams_ctx *c)
{
    double *E, *Fk, *G;
    int m, Z;
    blocktri_parts(c, E, Fk, G, m, Z);
    const int n = c->g.Nc, t = twist_plane(Z);
    const size_t mm = (size_t)m * m;
    const double *Ac = c->a.Ac;
    auto D = [&](int k) { return Ac + (size_t)k * m * n + (size_t)k * m; };
    auto Lo = [&](int k) { return Ac + (size_t)k * m * n + (size_t)(k - 1) * m; };
    auto Up = [&](int k) { return Ac + (size_t)k * m * n + (size_t)(k + 1) * m; };
    // column nonzeros (m x 9) of a coupling block, one buffer per chain
    double *const Uc[2] = {c->a.work, c->a.work + (size_t)9 * m};
    const int nbx = c->g.nb[0], nby = c->g.nb[1];
    const dim3 rows(cdiv(m, kBlock), m);
    const unsigned cols9 = cdiv((size_t)9 * m, kBlock), cells = cdiv(mm, kBlock);
    std::vector<double *> mats;
    std::vector<int> chains;
    for (int k = 0; k < Z; ++k) {
        mats.push_back(E + k * mm);
        chains.push_back(k > t ? 1 : 0);
    }
    gj_prepare(c, mats, chains, m);
    hipStream_t s0 = c->stream, s1 = c->side ? c->side : c->stream;
    if (s1 != s0) {
        CAMS_HIP(hipEventRecord(c->fork_ev, s0));
        CAMS_HIP(hipStreamWaitEvent(s1, c->fork_ev, 0));
    }
    // top chain, planes 0 .. t-1
    for (int k = 0; k < t; ++k) {
        double *S = E + k * mm;
        k_copy2d<<<cells, kBlock, 0, s0>>>(D(k), n, S, m, m, m);
        if (k > 0) {
            k_plane_left<<<rows, kBlock, 0, s0>>>(Fk + k * mm, Lo(k), n, E + (k - 1) * mm, m, nbx, nby);
            k_plane_cols<<<cols9, kBlock, 0, s0>>>(Uc[0], Up(k - 1), n, m, nbx, nby);
            k_plane_right<<<rows, kBlock, 0, s0>>>(S, Fk + k * mm, Uc[0], m, nbx, nby, 1);
        }
        inverse_gj(c, S, m, k, 0, s0);
        if (k > 0)   // G_{k-1} = E_{k-1} U_{k-1}
            k_plane_right<<<rows, kBlock, 0, s0>>>(G + (k - 1) * mm, E + (k - 1) * mm, Uc[0], m, nbx, nby, 0);
    }
    k_plane_cols<<<cols9, kBlock, 0, s0>>>(Uc[0], Up(t - 1), n, m, nbx, nby);
    k_plane_right<<<rows, kBlock, 0, s0>>>(G + (t - 1) * mm, E + (t - 1) * mm, Uc[0], m, nbx, nby, 0);
    k_plane_left<<<rows, kBlock, 0, s0>>>(Fk + t * mm, Lo(t), n, E + (t - 1) * mm, m, nbx, nby);
    // bottom chain, planes Z-1 .. t+1
    for (int k = Z - 1; k > t; --k) {
        double *S = E + k * mm;
        k_copy2d<<<cells, kBlock, 0, s1>>>(D(k), n, S, m, m, m);
        if (k < Z - 1) {
            k_plane_left<<<rows, kBlock, 0, s1>>>(Fk + (k + 1) * mm, Up(k), n, E + (k + 1) * mm, m, nbx, nby);
            k_plane_cols<<<cols9, kBlock, 0, s1>>>(Uc[1], Lo(k + 1), n, m, nbx, nby);
            k_plane_right<<<rows, kBlock, 0, s1>>>(S, Fk + (k + 1) * mm, Uc[1], m, nbx, nby, 1);
        }
        inverse_gj(c, S, m, k, 1, s1);
        if (k < Z - 1)   // K_{k+1} = E_{k+1} L_{k+1}
            k_plane_right<<<rows, kBlock, 0, s1>>>(G + (k + 1) * mm, E + (k + 1) * mm, Uc[1], m, nbx, nby, 0);
    }
    k_plane_cols<<<cols9, kBlock, 0, s1>>>(Uc[1], Lo(t + 1), n, m, nbx, nby);
    k_plane_right<<<rows, kBlock, 0, s1>>>(G + (t + 1) * mm, E + (t + 1) * mm, Uc[1], m, nbx, nby, 0);
    k_plane_left<<<rows, kBlock, 0, s1>>>(Fk + (t + 1) * mm, Up(t), n, E + (t + 1) * mm, m, nbx, nby);
    if (s1 != s0) {
        CAMS_HIP(hipEventRecord(c->join_ev, s1));
        CAMS_HIP(hipStreamWaitEvent(s0, c->join_ev, 0));
    }
    // twist plane
    double *S = E + t * mm;
    k_copy2d<<<cells, kBlock, 0, s0>>>(D(t), n, S, m, m, m);
    k_plane_cols<<<cols9, kBlock, 0, s0>>>(Uc[0], Up(t - 1), n, m, nbx, nby);
    k_plane_right<<<rows, kBlock, 0, s0>>>(S, Fk + t * mm, Uc[0], m, nbx, nby, 1);
    k_plane_cols<<<cols9, kBlock, 0, s0>>>(Uc[0], Lo(t + 1), n, m, nbx, nby);
    k_plane_right<<<rows, kBlock, 0, s0>>>(S, Fk + (t + 1) * mm, Uc[0], m, nbx, nby, 1);
    inverse_gj(c, S, m, t, 0, s0);
}

// xc = A_c^-1 rc by block substitution from both ends:
//   g_k = rc_k - F_k g_{k-1} (k = 1..t),  g_k = rc_k - H_k g_{k+1} (k = Z-2..t+1),
//   then g_t -= H_t g_{t+1};  x_k = E_k g_k for every plane;
//   x_k -= G_k x_{k+1} (k = t-1..0),  x_k -= K_k x_{k-1} (k = t+1..Z-1).
// The two chains go in pairs, one launch per step.  rc is overwritten by g.
static void solve_blocktri(cams_ctx *c, double *rc, double *xc, const int32_t *done)
{
    double *E, *Fk, *G;
    int m, Z;
    blocktri_parts(c, E, Fk, G, m, Z);
    const int t = twist_plane(Z);
    const size_t mm = (size_t)m * m;
    auto pair = [&](bool has0, GemvJob a, bool has1, GemvJob b) {
        if (!has0 && !has1) return;
        if (!has0) a = b;
        const int rows = (has0 && has1 ? 2 : 1) * m;
        k_gemv_pair<<<cdiv(rows, kBlock / 64), kBlock, 0, c->stream>>>(a, b, m, rows, done);
    };
    const int nt = t, nbm = Z - 2 - t;   // forward steps of each chain
    for (int i = 0; i < std::max(nt, nbm); ++i) {
        const int kt = 1 + i, kb = Z - 2 - i;
        pair(i < nt, GemvJob{Fk + kt * mm, rc + (size_t)(kt - 1) * m, rc + (size_t)kt * m, -1.0, 1.0},
             i < nbm, GemvJob{Fk + (kb + 1) * mm, rc + (size_t)(kb + 1) * m, rc + (size_t)kb * m, -1.0, 1.0});
    }
    pair(true, GemvJob{Fk + (t + 1) * mm, rc + (size_t)(t + 1) * m, rc + (size_t)t * m, -1.0, 1.0}, false,
         GemvJob{});
    k_gemv_planes<<<cdiv((size_t)Z * m, kBlock / 64), kBlock, 0, c->stream>>>(E, m, (size_t)Z * m, rc, xc, done);
    const int ut = t, ub = Z - 1 - t;    // backward steps of each chain
    for (int i = 0; i < std::max(ut, ub); ++i) {
        const int kt = t - 1 - i, kb = t + 1 + i;
        pair(i < ut, GemvJob{G + kt * mm, xc + (size_t)(kt + 1) * m, xc + (size_t)kt * m, -1.0, 1.0},
             i < ub, GemvJob{G + kb * mm, xc + (size_t)(kb - 1) * m, xc + (size_t)kb * m, -1.0, 1.0});
    }
}

void launch_coarse_factor(cams_ctx *c)
{
    const int n = c->g.Nc;
    double *F = c->a.work;
    const size_t nn = (size_t)n * n;
    const bool pivoting = c->opt.restriction != CAMS_R_FE;
    double *X = c->a.Ainv;
    if (c->blocktri) {
        factor_blocktri(c);
        return;
    }
    if (!pivoting) {   // Gauss-Jordan in place in X
        gj_prepare(c, {X}, {0}, n);
        k_copy<<<cdiv(nn, kBlock), kBlock, 0, c->stream>>>(c->a.Ac, X, nn);
        inverse_gj(c, X, n, 0, 0, c->stream);
        if (c->a.Ainv32) {
            const int T = (n + 63) / 64;
            k_round_lower<<<T * (T + 1) / 2, kBlock, 0, c->stream>>>(X, c->a.Ainv32, n);
            c->ainv32_ok = true;
        }
        return;
    }
    k_copy<<<cdiv(nn, kBlock), kBlock, 0, c->stream>>>(c->a.Ac, F, nn);
    // LU with partial pivoting, right looking by panels
    for (int j0 = 0; pivoting && j0 < n; j0 += kNB) {
        const int nb = n - j0 < kNB ? n - j0 : kNB;
        if ((size_t)(n - j0) * (nb + 1) <= (size_t)kPanelLds)
            k_lu_panel_lds<<<1, kBlock, 0, c->stream>>>(F, n, j0, nb, c->a.piv, c->a.status);
        else
            k_lu_panel<<<1, kBlock, 0, c->stream>>>(F, n, j0, nb, c->a.piv, c->a.status);
        if (n - nb > 0) k_lu_swap<<<cdiv(n - nb, kBlock), kBlock, 0, c->stream>>>(F, n, j0, nb, c->a.piv);
        const int rest = n - j0 - nb;
        if (rest > 0) {
            k_trsm<<<cdiv(rest, kBlock), kBlock, 0, c->stream>>>(F, n, j0, nb, F, n, j0 + nb, rest, 0);
            gemm_sub(c, F + (size_t)(j0 + nb) * n + j0 + nb, n, F + (size_t)(j0 + nb) * n + j0, n,
                     F + (size_t)j0 * n + j0 + nb, n, rest, rest, nb);
        }
    }
    // inverse: X = U^{-1} L^{-1} (P I)
    int32_t *perm = c->a.piv + n;
    k_perm_identity<<<1, 1, 0, c->stream>>>(c->a.piv, n, perm, X);
    k_perm_fill<<<cdiv(nn, kBlock), kBlock, 0, c->stream>>>(perm, n, X);
    for (int j0 = 0; j0 < n; j0 += kNB) {
        const int nb = n - j0 < kNB ? n - j0 : kNB;
        k_trsm<<<cdiv(n, kBlock), kBlock, 0, c->stream>>>(F, n, j0, nb, X, n, 0, n, 0);
        const int rest = n - j0 - nb;
        if (rest > 0)
            gemm_sub(c, X + (size_t)(j0 + nb) * n, n, F + (size_t)(j0 + nb) * n + j0, n, X + (size_t)j0 * n, n, rest,
                     n, nb);
    }
    const int last = ((n - 1) / kNB) * kNB;
    for (int j0 = last; j0 >= 0; j0 -= kNB) {
        const int nb = n - j0 < kNB ? n - j0 : kNB;
        k_trsm<<<cdiv(n, kBlock), kBlock, 0, c->stream>>>(F, n, j0, nb, X, n, 0, n, 1);
        if (j0 > 0) gemm_sub(c, X, n, F + j0, n, X + (size_t)j0 * n, n, j0, n, nb);
    }
}

// xc = A_c^-1 (R r) from the restriction slots.  With stop_parts > 0 the
// stopping test on that many residual partials runs first: inside the GEMV
// launch when the coarse system is small enough for the LDS form, else as a
// launch of its own.
void launch_gemv(cams_ctx *c, const double *rc, double *xc, const int32_t *done, int stop_parts)
{
    const int n = c->g.Nc;
    const int fe = c->opt.restriction == CAMS_R_FE;
    const double rt = c->opt.lin_rtol;
    if (!c->blocktri && n <= kGemvLds) {
        const bool stop = stop_parts > 0;
        k_gemv<<<cdiv(n, kBlock / 64) + (stop ? 1 : 0), kBlock, 0, c->stream>>>(
            c->a.Ainv, n, nullptr, c->g, c->a.slots, fe, xc, done, stop ? c->a.partial : nullptr, stop_parts,
            c->a.ictl, c->a.scal, rt * rt, c->opt.lin_maxit);
        return;
    }
    if (!c->blocktri && fe) {   // symmetric inverse: its lower triangle, once
        const int T = (n + 63) / 64;
        const bool stop = stop_parts > 0;
        const unsigned wgs = T * (T + 1) / 2 + (stop ? 1 : 0);
        if (c->a.Ainv32 && c->ainv32_ok)
            k_gemv_sym<float><<<wgs, kBlock, 0, c->stream>>>(c->a.Ainv32, n, c->g, c->a.slots, fe, c->a.rc, c->a.gpart,
                                                            done, stop ? c->a.partial : nullptr, stop_parts,
                                                            c->a.ictl, c->a.scal, rt * rt, c->opt.lin_maxit);
        else
            k_gemv_sym<double><<<wgs, kBlock, 0, c->stream>>>(c->a.Ainv, n, c->g, c->a.slots, fe, c->a.rc,
                                                             c->a.gpart, done, stop ? c->a.partial : nullptr,
                                                             stop_parts, c->a.ictl, c->a.scal, rt * rt,
                                                             c->opt.lin_maxit);
        k_gemv_sym_reduce<<<cdiv(n, kBlock), kBlock, 0, c->stream>>>(c->a.gpart, n, xc, done);
        return;
    }
    if (stop_parts > 0) launch_finalize_ctl(c, stop_parts);
    if (c->blocktri) {
        k_node_sum<<<cdiv(n, kBlock), kBlock, 0, c->stream>>>(c->g, c->a.slots, fe, c->a.rc, done);
        solve_blocktri(c, c->a.rc, xc, done);
    } else {
        k_node_sum<<<cdiv(n, kBlock), kBlock, 0, c->stream>>>(c->g, c->a.slots, fe, c->a.rc, done);
        k_gemv<<<cdiv(n, kBlock / 64), kBlock, 0, c->stream>>>(c->a.Ainv, n, c->a.rc, c->g, nullptr, fe, xc, done,
                                                             nullptr, 0, nullptr, nullptr, 0.0, 0);
    }
    (void)rc;
}

// xc = A_c^-1 rc for a given rc (test hook; rc is copied first).
void launch_coarse_solve(cams_ctx *c, const double *rc, double *xc)
{
    const int n = c->g.Nc;
    k_copy<<<cdiv(n, kBlock), kBlock, 0, c->stream>>>(rc, c->a.rc, (size_t)n);
    if (c->blocktri)
        solve_blocktri(c, c->a.rc, xc, nullptr);
    else
        k_gemv<<<cdiv(n, kBlock / 64), kBlock, 0, c->stream>>>(c->a.Ainv, n, c->a.rc, c->g, nullptr, 0, xc, nullptr,
                                                             nullptr, 0, nullptr, nullptr, 0.0, 0);
}

// Test hook: C -= A B on the device, same kernel as the factorisation.
void launch_gemm_sub(cams_ctx *c, double *C, int ldc, const double *A, int lda, const double *B, int ldb, int M,
                     int Nn, int K)
{
    gemm_sub(c, C, ldc, A, lda, B, ldb, M, Nn, K);
}

void launch_batch_node_sum(const BatchLaunch &L)
{
    launch_persistent(kb_node_sum, kBlock, L, L.inst, L.work, L.nwork);
}

void launch_batch_gemv(const BatchLaunch &L)
{
    launch_persistent(kb_gemv, kBlock, L, L.inst, L.work, L.nwork);
}

}  // namespace cams
