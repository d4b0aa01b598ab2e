// Natural-order (lexicographic) ILU(0) of the whole assembled matrix: the
// smoother of Table "cams" step 6 as the paper uses it (Sec. 3, Saad's
// ILU(0)).  For the 7-point operator in cell order ILU(0) drops no fill and
// changes only the diagonal, so with W the coupling magnitudes (A_mn = -W_mn,
// zero on every face of a well cell):
//   pivots   d_n = diag_n - sum_{m lower neighbour} W_mn^2 / d_m,
//   forward  y_n = (z_n + sum_{m lower} W_mn y_m) / d_n,
//   backward x_n = y_n + (sum_{m upper} W_nm x_m) / d_n,   x = M^{-1} z.
// Each recurrence is a wavefront: cell (i, j, k) needs only its three lower
// (upper) neighbours.  The grid is cut into 16 x 16 x 8 cell bricks (16 x 16
// x 1 on a 2D grid); the bricks of one diagonal bx + by + bz = s depend only
// on the diagonal before, so each diagonal is one launch with one workgroup
// per brick.  Inside a brick a thread owns a column (i, j) and walks it
// along z, taking cell (li, lj, lk) at step li + lj + lk: the x and y
// neighbours were finished one step earlier by the adjacent threads (read
// from the brick's result tile in LDS, one barrier per step), the z
// neighbour by the thread itself.  Values across brick faces come from the
// previous diagonal in global memory.  Operands are loaded all at once
// (branch-free, so every load is in flight together) and staged in LDS
// because a thread's step index differs from lane to lane; results leave
// the tile in one coalesced pass at the end.
#include "cams_internal.h"
#include "dev_util.h"

namespace cams {

namespace {

// Brick extent along x and y (one thread per column).  Measured on the
// 64x64x32 and 128^3 grids, 16 x 16 x 8 bricks beat single-wave 8 x 8 x 8
// ones by 1.05-1.17x per iteration: a diagonal's launch has a fixed cost
// (operand loads, stores, dispatch) of several microseconds, so fewer,
// longer diagonals win over shorter steps.
constexpr int kNatNB = 16;

// Bricks per axis and the brick depth along z.
struct NatGrid {
    int nb[3];
    int bz;
};

NatGrid nat_grid(const GridDev &g)
{
    constexpr int NB = kNatNB;
    NatGrid q;
    q.bz = g.nz > 1 ? 8 : 1;
    q.nb[0] = (g.nx + NB - 1) / NB;
    q.nb[1] = (g.ny + NB - 1) / NB;
    q.nb[2] = (g.nz + q.bz - 1) / q.bz;
    return q;
}

inline int nat_diagonals(const NatGrid &q) { return q.nb[0] + q.nb[1] + q.nb[2] - 2; }

// Bricks (bx, by, bz) on diagonal s, in order of bz, then by: within layer
// bz the rows by = first_row .. last_row (bx = s - bz - by).
__host__ __device__ __forceinline__ int first_row(const NatGrid &q, int s, int bz)
{
    const int v = s - bz - (q.nb[0] - 1);
    return v > 0 ? v : 0;
}
__host__ __device__ __forceinline__ int last_row(const NatGrid &q, int s, int bz)
{
    const int v = s - bz;
    return v < q.nb[1] - 1 ? v : q.nb[1] - 1;
}
__host__ __device__ __forceinline__ int first_layer(const NatGrid &q, int s)
{
    const int v = s - (q.nb[0] - 1) - (q.nb[1] - 1);
    return v > 0 ? v : 0;
}
__host__ __device__ __forceinline__ int last_layer(const NatGrid &q, int s)
{
    return s < q.nb[2] - 1 ? s : q.nb[2] - 1;
}

int bricks_on(const NatGrid &q, int s)
{
    int n = 0;
    for (int bz = first_layer(q, s); bz <= last_layer(q, s); ++bz) {
        const int c = last_row(q, s, bz) - first_row(q, s, bz) + 1;
        if (c > 0) n += c;
    }
    return n;
}

// Brick b of diagonal s (b below bricks_on(q, s)).
__device__ __forceinline__ void brick_at(const NatGrid &q, int s, int b, int &bx, int &by, int &bz)
{
    for (bz = first_layer(q, s); bz <= last_layer(q, s); ++bz) {
        const int lo = first_row(q, s, bz), c = last_row(q, s, bz) - lo + 1;
        if (c <= 0) continue;
        if (b < c) {
            by = lo + b;
            bx = s - bz - by;
            return;
        }
        b -= c;
    }
}

// Lower-triangular wavefront over one brick of diagonal s.
// MODE 0 (pivots): src = diag; writes invd[n] = 1 / d_n, reading invd of
//   finished neighbours (W^2 * invd = W^2 / d); a pivot that is not
//   positive raises F_BAD_PIVOT and is replaced by 1.
// MODE 1 (forward sweep): src = z; reads invd; writes y, reading y of
//   finished neighbours.
template <int NB, int BZ, int MODE>
__global__ __launch_bounds__(NB * NB) void k_nat_lower(GridDev g, NatGrid q, int s, const double *__restrict__ W,
                                                  const double *__restrict__ src, double *invd, double *y,
                                                  int32_t *status)
{
    constexpr int NT = NB * NB;
    constexpr int NA = MODE == 0 ? 4 : 5;   // staged operands: src, Wx-, Wy-, Wz- (, invd)
    constexpr int STEPS = 2 * (NB - 1) + BZ;
    __shared__ double opd[NA][BZ][NT];
    __shared__ double res[BZ][NT];
    __shared__ double hx[BZ][NB], hy[BZ][NB];
    int bx = 0, by = 0, bz = 0;
    brick_at(q, s, blockIdx.x, bx, by, bz);
    const int t = threadIdx.x, li = t % NB, lj = t / NB;
    const int i = bx * NB + li, j = by * NB + lj, k0 = bz * BZ;
    const int kn = g.nz - k0 < BZ ? g.nz - k0 : BZ;
    const bool on = i < g.nx && j < g.ny;
    const double *Wx = W, *Wy = W + g.N, *Wz = W + 2 * g.N;
    double *val = MODE == 0 ? invd : y;   // the recurrence's values
    const int n0 = i + g.nx * (j + g.ny * k0);
    // All loads first, from addresses kept inside the arrays (cell 0 stands
    // in for a missing neighbour or a cell outside the brick) and with no
    // branch between them, so that they are in flight together; the values
    // that do not exist are zeroed afterwards.
    double a[BZ], wx[BZ], wy[BZ], wz[BZ], id[BZ], hxv[BZ], hyv[BZ];
#pragma unroll
    for (int lk = 0; lk < BZ; ++lk) {
        const bool ok = on && lk < kn;
        const int n = ok ? n0 + lk * g.sxy : 0;
        a[lk] = src[n];
        id[lk] = MODE == 1 ? invd[n] : 0.0;
        wx[lk] = Wx[ok && i > 0 ? n - 1 : 0];
        wy[lk] = Wy[ok && j > 0 ? n - g.nx : 0];
        wz[lk] = Wz[ok && k0 + lk > 0 ? n - g.sxy : 0];
        // halo: the x neighbour for the threads of the brick's x face, the
        // y neighbour for those of its y face
        hxv[lk] = val[ok && li == 0 && i > 0 ? n - 1 : 0];
        hyv[lk] = val[ok && lj == 0 && j > 0 ? n - g.nx : 0];
    }
    double prev = val[on && k0 > 0 ? n0 - g.sxy : 0];   // the z neighbour below the brick
    if (!(on && k0 > 0)) prev = 0.0;
#pragma unroll
    for (int lk = 0; lk < BZ; ++lk) {
        const bool ok = on && lk < kn;
        opd[0][lk][t] = ok ? a[lk] : 0.0;
        opd[1][lk][t] = ok && i > 0 ? wx[lk] : 0.0;
        opd[2][lk][t] = ok && j > 0 ? wy[lk] : 0.0;
        opd[3][lk][t] = ok && k0 + lk > 0 ? wz[lk] : 0.0;
        if (MODE == 1) opd[NA - 1][lk][t] = ok ? id[lk] : 0.0;
        if (ok && li == 0) hx[lk][lj] = i > 0 ? hxv[lk] : 0.0;
        if (ok && lj == 0) hy[lk][li] = j > 0 ? hyv[lk] : 0.0;
    }
    __syncthreads();
    const int base = li + lj;
    for (int l = 0; l < STEPS; ++l) {
        const int lk = l - base;
        if (on && lk >= 0 && lk < kn) {
            const double vx = li > 0 ? res[lk][t - 1] : hx[lk][lj];
            const double vy = lj > 0 ? res[lk][t - NB] : hy[lk][li];
            const double a = opd[0][lk][t], wx = opd[1][lk][t], wy = opd[2][lk][t], wz = opd[3][lk][t];
            double v;
            if (MODE == 0) {
                double d = a - wx * wx * vx - wy * wy * vy - wz * wz * prev;
                if (!(d > 0.0)) {
                    atomicOr(status, F_BAD_PIVOT);
                    d = 1.0;
                }
                v = 1.0 / d;
            } else {
                v = (a + wx * vx + wy * vy + wz * prev) * opd[NA - 1][lk][t];
            }
            res[lk][t] = v;
            prev = v;
        }
        __syncthreads();
    }
    if (on)
#pragma unroll
        for (int lk = 0; lk < BZ; ++lk)
            if (lk < kn) val[n0 + lk * g.sxy] = res[lk][t];
}

// Backward sweep over one brick of diagonal s (diagonals taken from the
// last to the first): xy holds y on entry and x = M^{-1} z where finished;
// e = x (first step) or e + x.
template <int NB, int BZ>
__global__ __launch_bounds__(NB * NB) void k_nat_upper(GridDev g, NatGrid q, int s, const double *__restrict__ W,
                                                  const double *__restrict__ invd, double *xy,
                                                  double *__restrict__ e, int first)
{
    constexpr int NT = NB * NB;
    constexpr int STEPS = 2 * (NB - 1) + BZ;
    __shared__ double opd[5][BZ][NT];   // y, Wx+, Wy+, Wz+, invd
    __shared__ double res[BZ][NT];
    __shared__ double hx[BZ][NB], hy[BZ][NB];
    int bx = 0, by = 0, bz = 0;
    brick_at(q, s, blockIdx.x, bx, by, bz);
    const int t = threadIdx.x, li = t % NB, lj = t / NB;
    const int i = bx * NB + li, j = by * NB + lj, k0 = bz * BZ;
    const int kn = g.nz - k0 < BZ ? g.nz - k0 : BZ;
    const bool on = i < g.nx && j < g.ny;
    const bool xin = i + 1 < g.nx, yin = j + 1 < g.ny;   // upper x / y neighbour inside the grid
    const double *Wx = W, *Wy = W + g.N, *Wz = W + 2 * g.N;
    const int n0 = i + g.nx * (j + g.ny * k0);
    // loads first, branch-free from in-range addresses (as in k_nat_lower),
    // including the correction e that the end adds to
    double yv[BZ], wx[BZ], wy[BZ], wz[BZ], id[BZ], hxv[BZ], hyv[BZ], eo[BZ];
#pragma unroll
    for (int lk = 0; lk < BZ; ++lk) {
        const bool ok = on && lk < kn;
        const int n = ok ? n0 + lk * g.sxy : 0;
        yv[lk] = xy[n];
        id[lk] = invd[n];
        wx[lk] = Wx[n];
        wy[lk] = Wy[n];
        wz[lk] = Wz[n];
        eo[lk] = first ? 0.0 : e[n];
        hxv[lk] = xy[ok && li == NB - 1 && xin ? n + 1 : 0];
        hyv[lk] = xy[ok && lj == NB - 1 && yin ? n + g.nx : 0];
    }
    const bool above = on && k0 + kn < g.nz;
    double prev = xy[above ? n0 + kn * g.sxy : 0];   // the z neighbour above the brick
    if (!above) prev = 0.0;
#pragma unroll
    for (int lk = 0; lk < BZ; ++lk) {
        const bool ok = on && lk < kn;
        opd[0][lk][t] = ok ? yv[lk] : 0.0;
        opd[1][lk][t] = ok && xin ? wx[lk] : 0.0;
        opd[2][lk][t] = ok && yin ? wy[lk] : 0.0;
        opd[3][lk][t] = ok && k0 + lk + 1 < g.nz ? wz[lk] : 0.0;
        opd[4][lk][t] = ok ? id[lk] : 0.0;
        if (ok && li == NB - 1) hx[lk][lj] = xin ? hxv[lk] : 0.0;
        if (ok && lj == NB - 1) hy[lk][li] = yin ? hyv[lk] : 0.0;
    }
    __syncthreads();
    const int base = li + lj;
    for (int l = STEPS - 1; l >= 0; --l) {
        const int lk = l - base;
        if (on && lk >= 0 && lk < kn) {
            const double vx = li < NB - 1 ? (xin ? res[lk][t + 1] : 0.0) : hx[lk][lj];
            const double vy = lj < NB - 1 ? (yin ? res[lk][t + NB] : 0.0) : hy[lk][li];
            const double x = opd[0][lk][t] +
                             opd[4][lk][t] * (opd[1][lk][t] * vx + opd[2][lk][t] * vy + opd[3][lk][t] * prev);
            res[lk][t] = x;
            prev = x;
        }
        __syncthreads();
    }
    if (on)
#pragma unroll
        for (int lk = 0; lk < BZ; ++lk)
            if (lk < kn) {
                const int n = n0 + lk * g.sxy;
                const double x = res[lk][t];
                xy[n] = x;
                e[n] = eo[lk] + x;
            }
}

template <int NB, int BZ>
void nat_setup(cams_ctx *c, const NatGrid &q)
{
    const int L = nat_diagonals(q);
    for (int s = 0; s < L; ++s)
        k_nat_lower<NB, BZ, 0><<<bricks_on(q, s), NB * NB, 0, c->stream>>>(c->g, q, s, c->a.W, c->a.diag, c->a.invd,
                                                                   nullptr, c->a.status);
}

template <int NB, int BZ>
void nat_smooth(cams_ctx *c, const NatGrid &q, const double *rhs, double *e, int steps)
{
    const int L = nat_diagonals(q);
    for (int st = 0; st < steps; ++st) {
        const double *z = rhs;
        if (st > 0) {
            launch_stencil_sub(c, rhs, e, c->a.z, nullptr);   // z = rhs - A e
            z = c->a.z;
        }
        for (int s = 0; s < L; ++s)
            k_nat_lower<NB, BZ, 1><<<bricks_on(q, s), NB * NB, 0, c->stream>>>(c->g, q, s, c->a.W, z, c->a.invd, c->a.x,
                                                                       nullptr);
        for (int s = L - 1; s >= 0; --s)
            k_nat_upper<NB, BZ><<<bricks_on(q, s), NB * NB, 0, c->stream>>>(c->g, q, s, c->a.W, c->a.invd, c->a.x, e,
                                                                    st == 0);
    }
}

}  // namespace

void launch_nat_setup(cams_ctx *c)
{
    const NatGrid q = nat_grid(c->g);
    if (q.bz == 8)
        nat_setup<kNatNB, 8>(c, q);
    else
        nat_setup<kNatNB, 1>(c, q);
}

// e = sum of `steps` ILU(0)-preconditioned Richardson steps on A e = rhs from
// e = 0: e += M^{-1}(rhs - A e).  Host-controlled (no stop flag).
void launch_nat_smooth(cams_ctx *c, const double *rhs, double *e, int steps)
{
    const NatGrid q = nat_grid(c->g);
    if (q.bz == 8)
        nat_smooth<kNatNB, 8>(c, q, rhs, e, steps);
    else
        nat_smooth<kNatNB, 1>(c, q, rhs, e, steps);
}

}  // namespace cams
