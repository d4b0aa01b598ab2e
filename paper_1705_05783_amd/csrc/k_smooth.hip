// Block-Jacobi ILU(0) smoother (Table "cams" step 6: n_s ILU(0) smoothing
// steps).  The grid is cut into 8x8x8 cell blocks (8x8 in 2D; the last block
// of an axis may be shorter).  Couplings across block faces are left out of
// the factorisation, so every block is an independent ILU(0) in natural
// order that one wave solves in LDS by hyperplane wavefronts (i+j+k =
// const, 22 levels for a full block); the Richardson residual of each step
// still uses the full matrix.
//
// The alternating form takes every other step on a second block grid,
// shifted cyclically by half a block on every axis longer than one block
// (a shorter axis is one block either way): along x the block
// holds 8 consecutive positions p, cell i = (p - ox) mod nx.  The block that
// wraps round the end of an axis is two pieces with no coupling between
// them (the coupling of cell nx-1 to its +x side is the zero boundary
// face), so it is still one block of the same shape for the kernels; the
// faces the first grid leaves out are inside the blocks of the second.
//
// For the 7-point matrix in natural order ILU(0) keeps the off-diagonals of
// A and only modifies the diagonal: d_i = a_ii - sum_{j<i} W_ij^2 / d_j.
// One application of M^{-1} z is then
//   forward   y_i = (z_i + sum_{j<i} W_ij y_j) / d_i,
//   backward  x_i = y_i + (sum_{j>i} W_ij x_j) / d_i.
//
// Workgroups are mapped XCD-aware: consecutive logical blocks (neighbours
// along x, which share 128-byte lines of every array) are given to
// workgroup ids that the dispatcher sends to the same XCD, so the shared
// lines are fetched into one L2 instead of two.
#include <type_traits>

#include "cams_internal.h"
#include "dev_util.h"

namespace cams {

namespace {

constexpr int SB = 8;                 // block extent per active axis
constexpr int ST = SB * SB * SB;      // one thread per cell

struct BlockCell {
    int n;          // global cell index
    int t;          // local slot li + 8 lj + 64 lk
    int li, lj, lk;
    int ex, ey, ez; // block extents
    int i, j, k;
    bool active;
};

// Offsets of the shifted block grid: half a block on every axis longer than
// one block.  An axis of at most one block stays unshifted: its single block
// holds the whole axis either way, and the cyclic positions would put the
// grid neighbours at positions n-1 and 0 at the two ends of that block.
struct Shift {
    int x, y, z;
};

__device__ __forceinline__ Shift block_shift(const GridDev &g, int shifted)
{
    if (!shifted) return Shift{0, 0, 0};
    return Shift{g.nx > SB ? SB / 2 : 0, g.ny > SB ? SB / 2 : 0, g.nz > SB ? SB / 2 : 0};
}

// Cell coordinate of position p on an axis of n cells shifted by o < n.
__device__ __forceinline__ int wrap_cell(int p, int o, int n)
{
    const int i = p - o;
    return i < 0 ? i + n : i;
}

// Cell of this thread in logical block `id` (x fastest, then y, then z).
__device__ __forceinline__ BlockCell block_cell(const GridDev &g, int id, Shift o)
{
    BlockCell b;
    const int nbx = (g.nx + SB - 1) / SB, nby = (g.ny + SB - 1) / SB;
    const int bx = id % nbx, by = (id / nbx) % nby, bz = id / (nbx * nby);
    const int i0 = bx * SB, j0 = by * SB, k0 = bz * SB;
    b.ex = min(SB, g.nx - i0);
    b.ey = min(SB, g.ny - j0);
    b.ez = min(SB, g.nz - k0);
    b.t = threadIdx.x;
    b.li = b.t & (SB - 1);
    b.lj = (b.t >> 3) & (SB - 1);
    b.lk = b.t >> 6;
    b.active = b.li < b.ex && b.lj < b.ey && b.lk < b.ez;
    b.i = wrap_cell(i0 + b.li, o.x, g.nx);
    b.j = wrap_cell(j0 + b.lj, o.y, g.ny);
    b.k = wrap_cell(k0 + b.lk, o.z, g.nz);
    b.n = b.active ? b.i + g.nx * (b.j + g.ny * b.k) : 0;
    return b;
}

// Pivots of the block ILU(0), once per assembled matrix (`shifted`: on the
// shifted block grid).  A cell's lower neighbour in the block is its lower
// neighbour in the grid, except at the seam of a wrapped block (cell 0 after
// cell n-1), where the two are not coupled.
__global__ __launch_bounds__(ST) void k_bilu_setup(GridDev g, const double *__restrict__ W,
                                                    const double *__restrict__ diag, double *__restrict__ invd,
                                                    int32_t *status, int shifted)
{
    __shared__ double d[ST];
    const BlockCell b = block_cell(g, xcd_swizzle(blockIdx.x, gridDim.x), block_shift(g, shifted));
    const double *Wx = W, *Wy = W + g.N, *Wz = W + 2 * g.N;
    double dg = 1.0, wxm = 0.0, wym = 0.0, wzm = 0.0;
    if (b.active) {
        dg = diag[b.n];
        if (b.li > 0 && b.i > 0) wxm = Wx[b.n - 1];
        if (b.lj > 0 && b.j > 0) wym = Wy[b.n - g.nx];
        if (b.lk > 0 && b.k > 0) wzm = Wz[b.n - g.sxy];
    }
    d[b.t] = 1.0;
    __syncthreads();
    const int lev = b.li + b.lj + b.lk;
    const int nlev = b.ex + b.ey + b.ez - 2;
    for (int l = 0; l < nlev; ++l) {
        if (b.active && lev == l) {
            double v = dg;
            if (b.li > 0) v -= wxm * wxm / d[b.t - 1];
            if (b.lj > 0) v -= wym * wym / d[b.t - SB];
            if (b.lk > 0) v -= wzm * wzm / d[b.t - SB * SB];
            if (!(v > 0.0)) {
                atomicOr(status, F_BAD_PIVOT);
                v = 1.0;
            }
            d[b.t] = v;
        }
        __syncthreads();
    }
    if (b.active) invd[b.n] = 1.0 / d[b.t];
}

constexpr int PAD = SB * SB;

// One Richardson step  e_new = e_old + M^{-1}(rhs - A e_old)  (e_old = 0 when
// null) for logical block `blk` by a workgroup of NT threads (NT = 64..512,
// ST / NT cells per thread): all threads stage the block (residual with the
// full matrix, pivots, in-block couplings) into LDS; the first wave alone
// sweeps the hyperplanes forward and backward, one lane per x-pencil (only
// wave-level ordering inside the sweeps); then all threads write the block
// back.  Fewer threads per block let a compute unit keep more blocks, and so
// more of the latency-bound sweeps, in flight; the batched solve tunes NT.
//
// Two sweep forms, equal bit for bit:
//  SW = 0  the running values live in LDS: every level reads its
//          neighbours' results of the previous level back from LDS (little
//          register use, so many blocks per compute unit: grids with many
//          more blocks than compute units);
//  SW = 1  the running values live in registers: each lane loads the
//          coefficients of all levels of its pencil before the sweep (the
//          loads do not depend on the recurrence, so all are in flight
//          together) and takes the previous level's values of its -y/+y and
//          -z/+z neighbour pencils (lanes -/+1 and -/+8) by ds_bpermute; a
//          level is then two lane exchanges and four arithmetic operations
//          on the critical path instead of an LDS write and read.  It needs
//          about 230 registers per lane, so it pays when every block of the
//          grid is resident at once (one block per compute unit).
// e_old and e_new must be different arrays: neighbouring blocks read e_old
// across block faces.  T: arithmetic and storage of the smoother (double, or
// float in the mixed precision solve); TR: type of the right-hand side.
//
// y and the +x/+y/+z couplings carry SB*SB zero entries on both sides, so
// the sweeps read neighbours without bounds tests: a coupling that leaves
// the block (or the grid) is zero, and its partner value is finite.
template <class T>
struct SmoothLds {
    T y[ST + 2 * PAD], wx[ST + 2 * PAD], wy[ST + 2 * PAD], wz[ST + 2 * PAD], dinv[ST];
};

__device__ __forceinline__ void wave_sync()
{
    // LDS operations of one wave execute in order; keep the compiler from
    // moving the next step's reads above this step's writes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Synchronisation of the threads that share one block: the workgroup, or
// one wave when every wave of the workgroup has a block of its own (NT = 64).
template <int NT>
__device__ __forceinline__ void team_sync()
{
    if constexpr (NT == 64)
        wave_sync();
    else
        __syncthreads();
}

// Value of v in lane `src` of the wave.
template <class T>
__device__ __forceinline__ T lane_value(T v, int src)
{
    if constexpr (sizeof(T) == 4) {
        return __int_as_float(__builtin_amdgcn_ds_bpermute(4 * src, __float_as_int(v)));
    } else {
        const unsigned long long b = (unsigned long long)__double_as_longlong(v);
        const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(4 * src, (int)(unsigned)b);
        const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(4 * src, (int)(unsigned)(b >> 32));
        return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    }
}

// Forward and backward sweeps of the staged block by the first wave with the
// running values in registers (SW = 1 above).  Lane (pj, pk) = (lane % 8,
// lane / 8) owns the x-pencil; at level tau it handles li = tau - pj - pk.
// Coefficients are loaded in batches of CH levels (all 22 in FP32, 11 in
// FP64 to bound the register count); inactive lanes keep their running value
// and store into the upper zero pad, which nothing reads here.
template <class T, int CHF = 0>
__device__ __forceinline__ void sweep_registers(SmoothLds<T> &L, int ex, int ey, int ez, int lane)
{
    constexpr int NL = 3 * SB - 2;
    constexpr int CH = CHF > 0 ? CHF : (sizeof(T) == 4 ? NL : NL / 2);
    const int pj = lane & (SB - 1), pk = lane >> 3;
    const bool pencil = pj < ey && pk < ez;
    const int base = PAD + SB * pj + SB * SB * pk, s0 = pj + pk;
    const int junk = PAD + ST + lane;
    const int ym = lane > 0 ? lane - 1 : 0, zm = lane >= SB ? lane - SB : 0;
    const int yp = lane < 63 ? lane + 1 : 63, zp = lane < 64 - SB ? lane + SB : 63;
    T yv[NL];
    T run = 0;
#pragma unroll
    for (int c0 = 0; c0 < NL; c0 += CH) {
        T z[CH], cx[CH], cy[CH], cz[CH], di[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int t = base + min(max(c0 + q - s0, 0), SB - 1);
            z[q] = L.y[t];
            cx[q] = L.wx[t - 1];
            cy[q] = L.wy[t - SB];
            cz[q] = L.wz[t - SB * SB];
            di[q] = L.dinv[t - PAD];
        }
        __builtin_amdgcn_sched_barrier(0);   // keep the batch of loads ahead of the recurrence
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int a = c0 + q - s0;
            const bool act = pencil && a >= 0 && a < ex;
            const T s = z[q] + cx[q] * run + cy[q] * lane_value(run, ym) + cz[q] * lane_value(run, zm);
            const T v = s * di[q];
            run = act ? v : run;
            yv[c0 + q] = v;
        }
    }
    run = 0;
#pragma unroll
    for (int c0 = NL - CH; c0 >= 0; c0 -= CH) {
        T cx[CH], cy[CH], cz[CH], di[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int t = base + min(max(c0 + q - s0, 0), SB - 1);
            cx[q] = L.wx[t];
            cy[q] = L.wy[t];
            cz[q] = L.wz[t];
            di[q] = L.dinv[t - PAD];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = CH - 1; q >= 0; --q) {
            const int a = c0 + q - s0;
            const bool act = pencil && a >= 0 && a < ex;
            const int t = base + min(max(a, 0), SB - 1);
            const T s = cx[q] * run + cy[q] * lane_value(run, yp) + cz[q] * lane_value(run, zp);
            const T v = yv[c0 + q] + s * di[q];
            run = act ? v : run;
            L.y[act ? t : junk] = v;
        }
    }
}

// Forward and backward sweeps of the staged block by one wave with the
// running values in LDS (SW = 0): lane owns the x-pencil (pj, pk) =
// (lane % 8, lane / 8); at time step tau it handles the cell
// li = tau - pj - pk of hyperplane tau.
template <class T>
__device__ __forceinline__ void sweep_lds(SmoothLds<T> &L, int ex, int ey, int ez, int lane)
{
    T *y = L.y, *wx = L.wx, *wy = L.wy, *wz = L.wz, *dinv = L.dinv;
    const int pj = lane & (SB - 1), pk = lane >> 3;
    const bool pencil = pj < ey && pk < ez;
    const int nlev = ex + ey + ez - 2;
    const int base = PAD + SB * pj + SB * SB * pk;
    for (int tau = 0; tau < nlev; ++tau) {
        const int a = tau - pj - pk;
        const bool act = pencil && a >= 0 && a < ex;
        const int t = base + min(max(a, 0), SB - 1);
        const T s = y[t] + wx[t - 1] * y[t - 1] + wy[t - SB] * y[t - SB] + wz[t - SB * SB] * y[t - SB * SB];
        if (act) y[t] = s * dinv[t - PAD];
        wave_sync();
    }
    for (int tau = nlev - 1; tau >= 0; --tau) {
        const int a = tau - pj - pk;
        const bool act = pencil && a >= 0 && a < ex;
        const int t = base + min(max(a, 0), SB - 1);
        const T s = wx[t] * y[t + 1] + wy[t] * y[t + SB] + wz[t] * y[t + SB * SB];
        if (act) y[t] += s * dinv[t - PAD];
        wave_sync();
    }
}

// The LDS of one block for the row form, without the zero borders (10 KB
// in FP32, so that four workgroups of four blocks, 160 KB, share one
// compute unit and a 128^3 grid's 1024 workgroups run in one round instead
// of 1.33).  The sweeps clamp neighbour indices into the block: a coupling
// that leaves the block through a face inside it is zero in the arrays
// (staged so), and only those that leave through the block's first cell,
// first row or first layer (index below 0) are zeroed by a test; the
// partner values read there are finite.  The arithmetic equals sweep_lds.
template <class T>
struct SmoothLdsTight {
    T y[ST], wx[ST], wy[ST], wz[ST], dinv[ST];
};

template <class T>
__device__ __forceinline__ void sweep_lds_tight(SmoothLdsTight<T> &L, int ex, int ey, int ez, int lane)
{
    T *y = L.y, *wx = L.wx, *wy = L.wy, *wz = L.wz, *dinv = L.dinv;
    const int pj = lane & (SB - 1), pk = lane >> 3;
    const bool pencil = pj < ey && pk < ez;
    const int nlev = ex + ey + ez - 2;
    const int base = SB * pj + SB * SB * pk;
    for (int tau = 0; tau < nlev; ++tau) {
        const int a = tau - pj - pk;
        const bool act = pencil && a >= 0 && a < ex;
        const int t = base + min(max(a, 0), SB - 1);
        const int tx = max(t - 1, 0), ty = max(t - SB, 0), tz = max(t - SB * SB, 0);
        const T cx = wx[tx], cy = wy[ty], cz = wz[tz];
        const T s = y[t] + (t >= 1 ? cx : T(0)) * y[tx] + (t >= SB ? cy : T(0)) * y[ty] +
                    (t >= SB * SB ? cz : T(0)) * y[tz];
        if (act) y[t] = s * dinv[t];
        wave_sync();
    }
    for (int tau = nlev - 1; tau >= 0; --tau) {
        const int a = tau - pj - pk;
        const bool act = pencil && a >= 0 && a < ex;
        const int t = base + min(max(a, 0), SB - 1);
        const T s = wx[t] * y[min(t + 1, ST - 1)] + wy[t] * y[min(t + SB, ST - 1)] + wz[t] * y[min(t + SB * SB, ST - 1)];
        if (act) y[t] += s * dinv[t];
        wave_sync();
    }
}

// Prolongated coarse correction as e_old (the first post-smoothing step):
// basis P (TP = double, float or bfloat16 bits), Dirichlet mask, coarse
// solution, and an LDS cube of (SB + 2)^3 values for the block and its face
// neighbours.
template <class T, class TP>
struct FromCoarse {
    const TP *P;
    const uint8_t *dm;
    const double *xc;
    T *cube;
    double *xs;   // LDS room for kXcLds coarse values
};

constexpr int CB = SB + 2;    // cube edge: the block with one layer around it
constexpr int kXcLds = 2048;  // coarse vectors up to this size are copied into LDS by the first step

// e_old = P xc on the block's cells and on the cells across its six faces
// (those outside the grid get 0), into the LDS cube at (li+1, lj+1, lk+1).
// Split in two so that the caller can issue every load of the step before
// the first wait: cube_load gathers each slot's mask, node tables and basis
// values; cube_fill combines them with the coarse values (read from `xcs`,
// an LDS copy of xc when it fits) and stores the cube.
constexpr int kCubeSlots = ST + 6 * PAD;

template <int NT>
__device__ __forceinline__ void cube_slot(int q, int ex, int ey, int ez, int &ci, int &cj, int &ck, bool &need)
{
    ci = cj = ck = 0;
    need = false;
    if (q < ST) {
        ci = q & (SB - 1);
        cj = (q >> 3) & (SB - 1);
        ck = q >> 6;
        need = ci < ex && cj < ey && ck < ez;
    } else if (q < kCubeSlots) {
        const int f = (q - ST) >> 6, u = (q - ST) & (SB - 1), v = ((q - ST) >> 3) & (SB - 1);
        switch (f) {
        case 0: ci = -1; cj = u; ck = v; need = u < ey && v < ez; break;
        case 1: ci = ex; cj = u; ck = v; need = u < ey && v < ez; break;
        case 2: ci = u; cj = -1; ck = v; need = u < ex && v < ez; break;
        case 3: ci = u; cj = ey; ck = v; need = u < ex && v < ez; break;
        case 4: ci = u; cj = v; ck = -1; need = u < ex && v < ey; break;
        default: ci = u; cj = v; ck = ez; need = u < ex && v < ey; break;
        }
    }
}

template <class TP, int NT>
struct CubeLoads {
    static constexpr int R = (kCubeSlots + NT - 1) / NT;
    ProlongIn<TP> in[R];
    int idx[R];
    bool need[R], inside[R];
};

template <class T, class TP, int NT>
__device__ __forceinline__ void cube_load(const GridDev &g, const FromCoarse<T, TP> &fc, int i0, int j0, int k0,
                                          int ex, int ey, int ez, CubeLoads<TP, NT> &cl, int tid)
{
#pragma unroll
    for (int h = 0; h < CubeLoads<TP, NT>::R; ++h) {
        int ci, cj, ck;
        bool need;
        cube_slot<NT>(tid + h * NT, ex, ey, ez, ci, cj, ck, need);
        const int i = i0 + ci, j = j0 + cj, k = k0 + ck;
        const bool in = need && i >= 0 && i < g.nx && j >= 0 && j < g.ny && k >= 0 && k < g.nz;
        const int ii = in ? i : i0, jj = in ? j : j0, kk = in ? k : k0;
        cl.in[h] = prolong_load(g, fc.P, fc.dm, ii + g.nx * (jj + g.ny * kk), ii, jj, kk);
        cl.idx[h] = (ci + 1) + CB * (cj + 1) + CB * CB * (ck + 1);
        cl.need[h] = need;
        cl.inside[h] = in;
    }
}

template <class T, class TP, int NT>
__device__ __forceinline__ void cube_fill(const GridDev &g, const FromCoarse<T, TP> &fc,
                                          const CubeLoads<TP, NT> &cl, const double *xcs)
{
#pragma unroll
    for (int h = 0; h < CubeLoads<TP, NT>::R; ++h) {
        const T v = (T)prolong_combine(g, cl.in[h], xcs);
        if (cl.need[h]) fc.cube[cl.idx[h]] = cl.inside[h] ? v : T(0);
    }
}

// `o`: offsets of the block grid (the prolongating first step takes the
// grid at the origin only).  i0, j0, k0 are positions on the shifted axes.
template <class T, class TR, int NT, int SW = 0, class TP = void, int CHF = 0>
__device__ __forceinline__ void bilu_step_body(const GridDev &g, const T *__restrict__ W, const T *__restrict__ diag,
                                               const T *__restrict__ invd, const TR *__restrict__ rhs,
                                               const T *__restrict__ eold, T *__restrict__ enew, int blk,
                                               SmoothLds<T> &L, Shift o, FromCoarse<T, TP> fc, int tid)
{
    constexpr int CPT = ST / NT;   // cells per thread
    const int nbx = (g.nx + SB - 1) / SB, nby = (g.ny + SB - 1) / SB;
    const int i0 = (blk % nbx) * SB, j0 = ((blk / nbx) % nby) * SB, k0 = (blk / (nbx * nby)) * SB;
    const int ex = min(SB, g.nx - i0), ey = min(SB, g.ny - j0), ez = min(SB, g.nz - k0);
    const T *Wx = W, *Wy = W + g.N, *Wz = W + 2 * g.N;
    for (int q = tid; q < 2 * PAD; q += NT) {
        const int idx = q < PAD ? q : ST + q;
        L.y[idx] = 0;
        L.wx[idx] = 0;
        L.wy[idx] = 0;
        L.wz[idx] = 0;
    }
    // Branch-free staging, so that all loads of a thread go out together:
    // slots outside a ragged block read the block's first cell and store
    // zeros; a neighbour outside the grid is the cell itself with coupling 0
    // (ae - 0 * e = ae).
    T e0[CPT];
    if constexpr (!std::is_void_v<TP>) {
        // e_old = P xc: the coefficient loads go out first, then the
        // prolongation fills the cube, then the residual reads e_old there
        T f6[CPT][6], dg[CPT], rh[CPT], idv[CPT];
        int qc[CPT];
        bool av[CPT];
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int t = tid + NT * c;
            const int li = t & (SB - 1), lj = (t >> 3) & (SB - 1), lk = t >> 6;
            const bool act = li < ex && lj < ey && lk < ez;
            const int ai = act ? li : 0, aj = act ? lj : 0, ak = act ? lk : 0;
            const int i = i0 + ai, j = j0 + aj, k = k0 + ak;
            const int n = i + g.nx * (j + g.ny * k);
            const bool xm = i > 0, xp = i + 1 < g.nx, ym = j > 0, yp = j + 1 < g.ny, zm = k > 0, zp = k + 1 < g.nz;
            const int nxm = xm ? n - 1 : n, nym = ym ? n - g.nx : n, nzm = zm ? n - g.sxy : n;
            const T wxm = Wx[nxm], wxp = Wx[n], wym = Wy[nym], wyp = Wy[n], wzm = Wz[nzm], wzp = Wz[n];
            f6[c][0] = xm ? wxm : T(0);
            f6[c][1] = xp ? wxp : T(0);
            f6[c][2] = ym ? wym : T(0);
            f6[c][3] = yp ? wyp : T(0);
            f6[c][4] = zm ? wzm : T(0);
            f6[c][5] = zp ? wzp : T(0);
            dg[c] = diag[n];
            rh[c] = (T)rhs[n];
            idv[c] = invd[n];
            qc[c] = (ai + 1) + CB * (aj + 1) + CB * CB * (ak + 1);
            av[c] = act;
        }
        // every global load of the step goes out here: the prolongation's
        // tables and basis values, and the coarse vector (into LDS when it fits)
        CubeLoads<TP, NT> cl;
        cube_load<T, TP, NT>(g, fc, i0, j0, k0, ex, ey, ez, cl, tid);
        const bool xlds = g.Nc <= kXcLds;
        if (xlds) {
            constexpr int XR = (kXcLds + NT - 1) / NT;
            double xv[XR];
#pragma unroll
            for (int h = 0; h < XR; ++h) {
                const int q = tid + h * NT;
                xv[h] = q < g.Nc ? fc.xc[q] : 0.0;
            }
#pragma unroll
            for (int h = 0; h < XR; ++h) {
                const int q = tid + h * NT;
                if (q < g.Nc) fc.xs[q] = xv[h];
            }
            team_sync<NT>();
        }
        cube_fill<T, TP, NT>(g, fc, cl, xlds ? fc.xs : fc.xc);
        team_sync<NT>();
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int t = tid + NT * c;
            const int li = t & (SB - 1), lj = (t >> 3) & (SB - 1), lk = t >> 6;
            const T *cb = fc.cube + qc[c];
            const T ec = cb[0];
            T ae = dg[c] * ec;
            ae -= f6[c][0] * cb[-1];
            ae -= f6[c][1] * cb[1];
            ae -= f6[c][2] * cb[-CB];
            ae -= f6[c][3] * cb[CB];
            ae -= f6[c][4] * cb[-CB * CB];
            ae -= f6[c][5] * cb[CB * CB];
            const bool act = av[c];
            e0[c] = act ? ec : T(0);
            L.y[PAD + t] = act ? rh[c] - ae : T(0);
            L.dinv[t] = act ? idv[c] : T(0);
            L.wx[PAD + t] = act && li + 1 < ex ? f6[c][1] : T(0);
            L.wy[PAD + t] = act && lj + 1 < ey ? f6[c][3] : T(0);
            L.wz[PAD + t] = act && lk + 1 < ez ? f6[c][5] : T(0);
        }
    } else {
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int t = tid + NT * c;
        const int li = t & (SB - 1), lj = (t >> 3) & (SB - 1), lk = t >> 6;
        const bool act = li < ex && lj < ey && lk < ez;
        const int i = wrap_cell(i0 + (act ? li : 0), o.x, g.nx), j = wrap_cell(j0 + (act ? lj : 0), o.y, g.ny);
        const int k = wrap_cell(k0 + (act ? lk : 0), o.z, g.nz);
        const int n = i + g.nx * (j + g.ny * k);
        const bool xm = i > 0, xp = i + 1 < g.nx, ym = j > 0, yp = j + 1 < g.ny, zm = k > 0, zp = k + 1 < g.nz;
        const int nxm = xm ? n - 1 : n, nxp = xp ? n + 1 : n, nym = ym ? n - g.nx : n, nyp = yp ? n + g.nx : n;
        const int nzm = zm ? n - g.sxy : n, nzp = zp ? n + g.sxy : n;
        const T wxm = Wx[nxm], wxp = Wx[n], wym = Wy[nym], wyp = Wy[n], wzm = Wz[nzm], wzp = Wz[n];
        const T fxm = xm ? wxm : T(0), fxp = xp ? wxp : T(0);
        const T fym = ym ? wym : T(0), fyp = yp ? wyp : T(0);
        const T fzm = zm ? wzm : T(0), fzp = zp ? wzp : T(0);
        // without e_old (a step from zero) the loads read W and the result is unused
        const T *eo = eold ? eold : W;
        const T ec = eo[n], exm = eo[nxm], exp = eo[nxp], eym = eo[nym], eyp = eo[nyp];
        const T ezm = eo[nzm], ezp = eo[nzp];
        T ae = diag[n] * ec;
        ae -= fxm * exm;
        ae -= fxp * exp;
        ae -= fym * eym;
        ae -= fyp * eyp;
        ae -= fzm * ezm;
        ae -= fzp * ezp;
        // weights instead of selects keep the compiler from splitting the code
        // on e_old (rhs - 1 * ae rounds as rhs - ae; rhs - 0 * ae = rhs)
        const T on = eold ? T(1) : T(0);
        const T z = (T)rhs[n] - on * ae;
        const T ev = on * ec;
        const T id = invd[n];
        e0[c] = act ? ev : T(0);
        L.y[PAD + t] = act ? z : T(0);
        L.dinv[t] = act ? id : T(0);
        // coupling to the +x/+y/+z neighbour when it lies in the block
        L.wx[PAD + t] = act && li + 1 < ex ? fxp : T(0);
        L.wy[PAD + t] = act && lj + 1 < ey ? fyp : T(0);
        L.wz[PAD + t] = act && lk + 1 < ez ? fzp : T(0);
    }
    }
    team_sync<NT>();
    if (SW == 1 && tid < 64) {
        sweep_registers<T, CHF>(L, ex, ey, ez, tid);
    } else if (SW == 0 && tid < 64) {
        sweep_lds<T>(L, ex, ey, ez, tid);
    }
    team_sync<NT>();
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int t = tid + NT * c;
        const int li = t & (SB - 1), lj = (t >> 3) & (SB - 1), lk = t >> 6;
        if (li < ex && lj < ey && lk < ez)
            enew[wrap_cell(i0 + li, o.x, g.nx) +
                 g.nx * (wrap_cell(j0 + lj, o.y, g.ny) + g.ny * wrap_cell(k0 + lk, o.z, g.nz))] =
                e0[c] + L.y[PAD + t];
    }
}

// Single-problem smoother: register sweeps with one 512-thread workgroup per
// block when all blocks are resident at once, else LDS sweeps with 256
// threads per block (several blocks per compute unit).
constexpr int kSmoothThreads = ST;
constexpr int kSmoothThreadsMany = 256;

template <class T, class TR, int NT, int SW>
__global__ __launch_bounds__(NT) void k_bilu_step(GridDev g, const T *__restrict__ W, const T *__restrict__ diag,
                                                   const T *__restrict__ invd, const TR *__restrict__ rhs,
                                                   const T *__restrict__ eold, T *__restrict__ enew,
                                                   const int32_t *done, int shifted)
{
    __shared__ SmoothLds<T> lds;
    if (done && *done) return;
    bilu_step_body<T, TR, NT, SW>(g, W, diag, invd, rhs, eold, enew, xcd_swizzle(blockIdx.x, gridDim.x), lds,
                                  block_shift(g, shifted), FromCoarse<T, void>{}, (int)threadIdx.x);
}

constexpr int kRowBlocks = 4;     // FP32 blocks per workgroup of the row form
constexpr int kRowThreads = 512;

// The same step for BPX neighbouring blocks along x per workgroup of NT
// threads: all threads stage the BPX blocks together, x fastest over the
// BPX * 8 cells of a row, so that a wave's loads cover rows of 8 BPX
// consecutive cells (128 bytes: BPX = 4 in FP32, 2 in FP64) instead of the
// 8-cell rows of one block; then wave w < BPX sweeps block w (those waves
// at once) and all threads write the blocks back.  The operations per cell
// are those of bilu_step_body.
// Group sb of BPX blocks along x (groups x fastest, then y, then z), as
// k_bilu_step_row and its batched form take it.  Each thread stages and
// writes back only its own LDS slots, so consecutive groups need no
// barrier between them.  LS: the block LDS with zero borders (SmoothLds)
// or without (SmoothLdsTight, swept by sweep_lds_tight).
template <class T, class TR, int BPX, int NT, class LS>
__device__ __forceinline__ void row_step_body(const GridDev &g, const T *__restrict__ W, const T *__restrict__ diag,
                                              const T *__restrict__ invd, const TR *__restrict__ rhs,
                                              const T *__restrict__ eold, T *__restrict__ enew, int sb, LS *Ls,
                                              Shift o, int tid)
{
    static_assert(NT % 64 == 0 && NT >= 64 * BPX && (ST * BPX) % NT == 0, "one wave per block at least");
    constexpr bool TIGHT = std::is_same<LS, SmoothLdsTight<T>>::value;
    constexpr int RX = SB * BPX, CPT = ST * BPX / NT, OFF = TIGHT ? 0 : PAD;
    if constexpr (!TIGHT) {
        for (int q = tid; q < BPX * 2 * PAD; q += NT) {
            const int b = q / (2 * PAD), r = q % (2 * PAD);
            const int idx = r < PAD ? r : ST + r;
            Ls[b].y[idx] = 0;
            Ls[b].wx[idx] = 0;
            Ls[b].wy[idx] = 0;
            Ls[b].wz[idx] = 0;
        }
    }
    const int nbx = (g.nx + SB - 1) / SB, nby = (g.ny + SB - 1) / SB;
    const int nsx = (nbx + BPX - 1) / BPX;
    const int bx0 = (sb % nsx) * BPX, j0 = ((sb / nsx) % nby) * SB, k0 = (sb / (nsx * nby)) * SB;
    const int ey = min(SB, g.ny - j0), ez = min(SB, g.nz - k0);
    const T *Wx = W, *Wy = W + g.N, *Wz = W + 2 * g.N;
    T e0[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int q = tid + NT * c;
        const int lx = q % RX, lj = (q / RX) % SB, lk = q / (RX * SB);
        const int b = lx / SB, li = lx % SB;
        const int i0 = (bx0 + b) * SB;
        const int ex = bx0 + b < nbx ? min(SB, g.nx - i0) : 0;
        const bool act = li < ex && lj < ey && lk < ez;
        const int i = act ? wrap_cell(i0 + li, o.x, g.nx) : 0;
        const int j = wrap_cell(j0 + (act ? lj : 0), o.y, g.ny), k = wrap_cell(k0 + (act ? lk : 0), o.z, g.nz);
        const int n = i + g.nx * (j + g.ny * k);
        const bool xm = i > 0, xp = i + 1 < g.nx, ym = j > 0, yp = j + 1 < g.ny, zm = k > 0, zp = k + 1 < g.nz;
        const int nxm = xm ? n - 1 : n, nxp = xp ? n + 1 : n, nym = ym ? n - g.nx : n, nyp = yp ? n + g.nx : n;
        const int nzm = zm ? n - g.sxy : n, nzp = zp ? n + g.sxy : n;
        const T wxm = Wx[nxm], wxp = Wx[n], wym = Wy[nym], wyp = Wy[n], wzm = Wz[nzm], wzp = Wz[n];
        const T fxm = xm ? wxm : T(0), fxp = xp ? wxp : T(0);
        const T fym = ym ? wym : T(0), fyp = yp ? wyp : T(0);
        const T fzm = zm ? wzm : T(0), fzp = zp ? wzp : T(0);
        const T *eo = eold ? eold : W;
        const T ec = eo[n], exm = eo[nxm], exp = eo[nxp], eym = eo[nym], eyp = eo[nyp];
        const T ezm = eo[nzm], ezp = eo[nzp];
        T ae = diag[n] * ec;
        ae -= fxm * exm;
        ae -= fxp * exp;
        ae -= fym * eym;
        ae -= fyp * eyp;
        ae -= fzm * ezm;
        ae -= fzp * ezp;
        const T on = eold ? T(1) : T(0);
        const T z = (T)rhs[n] - on * ae;
        const T ev = on * ec;
        const T id = invd[n];
        const int t = li + SB * lj + SB * SB * lk;
        LS &L = Ls[b];
        e0[c] = act ? ev : T(0);
        L.y[OFF + t] = act ? z : T(0);
        L.dinv[t] = act ? id : T(0);
        L.wx[OFF + t] = act && li + 1 < ex ? fxp : T(0);
        L.wy[OFF + t] = act && lj + 1 < ey ? fyp : T(0);
        L.wz[OFF + t] = act && lk + 1 < ez ? fzp : T(0);
    }
    __syncthreads();
    {
        const int w = tid >> 6;
        if (w < BPX && bx0 + w < nbx) {
            if constexpr (TIGHT)
                sweep_lds_tight<T>(Ls[w], min(SB, g.nx - (bx0 + w) * SB), ey, ez, tid & 63);
            else
                sweep_lds<T>(Ls[w], min(SB, g.nx - (bx0 + w) * SB), ey, ez, tid & 63);
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int q = tid + NT * c;
        const int lx = q % RX, lj = (q / RX) % SB, lk = q / (RX * SB);
        const int b = lx / SB, li = lx % SB;
        const int i0 = (bx0 + b) * SB;
        const int ex = bx0 + b < nbx ? min(SB, g.nx - i0) : 0;
        if (li < ex && lj < ey && lk < ez)
            enew[wrap_cell(i0 + li, o.x, g.nx) +
                 g.nx * (wrap_cell(j0 + lj, o.y, g.ny) + g.ny * wrap_cell(k0 + lk, o.z, g.nz))] =
                e0[c] + Ls[b].y[OFF + li + SB * lj + SB * SB * lk];
    }
}

// One round: the LDS without zero borders (40 KB) and at most 64 registers,
// four workgroups per compute unit, for grids whose groups all fit at once
// that way (128^3: 1024 groups, 22.6 -> 21.3 us per step).
template <class T, class TR, int BPX, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8))) void k_bilu_step_row(
    GridDev g, const T *__restrict__ W, const T *__restrict__ diag, const T *__restrict__ invd,
    const TR *__restrict__ rhs, const T *__restrict__ eold, T *__restrict__ enew, const int32_t *done, int shifted)
{
    __shared__ SmoothLdsTight<T> Ls[BPX];
    if (done && *done) return;
    row_step_body<T, TR, BPX, NT>(g, W, diag, invd, rhs, eold, enew, xcd_swizzle(blockIdx.x, gridDim.x), Ls,
                                  block_shift(g, shifted), (int)threadIdx.x);
}

// Several rounds: the LDS with zero borders and no register limit, whose
// staging keeps more loads in flight (256x256x128: 73 against 80 us for the
// one-round form).
template <class T, class TR, int BPX, int NT>
__global__ __launch_bounds__(NT) void k_bilu_step_rows(GridDev g, const T *__restrict__ W, const T *__restrict__ diag,
                                                        const T *__restrict__ invd, const TR *__restrict__ rhs,
                                                        const T *__restrict__ eold, T *__restrict__ enew,
                                                        const int32_t *done, int shifted)
{
    __shared__ SmoothLds<T> Ls[BPX];
    if (done && *done) return;
    row_step_body<T, TR, BPX, NT>(g, W, diag, invd, rhs, eold, enew, xcd_swizzle(blockIdx.x, gridDim.x), Ls,
                                  block_shift(g, shifted), (int)threadIdx.x);
}

// The first post-smoothing step, whose e_old is the prolongated coarse
// correction P xc (Eq. (12)): the prolongation runs inside the step (on the
// block and its face neighbours), so it needs no launch of its own and the
// correction d1 is never stored; the result equals prolongation followed by
// k_bilu_step bit for bit.
template <class T, class TR, int NT, int SW, class TP>
__global__ __launch_bounds__(NT) void k_bilu_first(GridDev g, const T *__restrict__ W, const T *__restrict__ diag,
                                                    const T *__restrict__ invd, const TR *__restrict__ rhs,
                                                    const TP *__restrict__ P, const uint8_t *__restrict__ dm,
                                                    const double *__restrict__ xc, T *__restrict__ enew,
                                                    const int32_t *done)
{
    __shared__ SmoothLds<T> lds;
    __shared__ T cube[CB * CB * CB];
    __shared__ double xs[kXcLds];
    if (done && *done) return;
    bilu_step_body<T, TR, NT, SW, TP>(g, W, diag, invd, rhs, nullptr, enew, xcd_swizzle(blockIdx.x, gridDim.x), lds,
                                      Shift{0, 0, 0}, FromCoarse<T, TP>{P, dm, xc, cube, xs}, (int)threadIdx.x);
}

// Batched step `s` of `steps` for every instance.  `post` selects the
// correction: post-smoothing writes d2 starting from d1 (so d2 ends as
// d1 + the smoothing correction), pre-smoothing writes d0 from zero.  The
// right-hand side is r, in the mixed-precision post-smoothing its FP32 copy.
// The work list is ordered host-side so that each XCD receives a contiguous
// range of logical blocks.
template <class T, class TR, int NT>
__global__ __launch_bounds__(NT) void kb_bilu_step(const InstDev *__restrict__ inst, const WorkItem *__restrict__ work,
                                                    const int32_t *nwork, int post, int s, int steps)
{
    __shared__ SmoothLds<T> lds;
    // each workgroup takes items blockIdx.x, + gridDim.x, ...; the next
    // item's descriptor is loaded while the current one runs
    const int nw = *nwork;
    int t = blockIdx.x;
    WorkItem wnext = t < nw ? work[t] : WorkItem{0, 0};
    for (; t < nw; t += gridDim.x) {
        const WorkItem w = wnext;
        if (t + (int)gridDim.x < nw) wnext = work[t + gridDim.x];
        const InstDev &d = inst[w.inst];
        if (d.a.ictl[C_DONE]) continue;
        const Arrays &a = d.a;
        const int shifted = d.alt && (s & 1);   // alternating smoother: odd steps on the shifted grid
        const T *W, *diag, *invd;
        T *e, *scratch;
        if constexpr (sizeof(T) == 4) {
            W = a.W32; diag = a.diag32; invd = a.invd32; e = post ? a.d2f : a.d0f; scratch = a.zf;
        } else {
            W = a.W; diag = a.diag; invd = a.invd; e = post ? a.d2 : a.d0; scratch = a.z;
        }
        const TR *rhs;
        if constexpr (sizeof(TR) == 4)
            rhs = a.r1f;
        else
            rhs = a.r;
        const T *init;   // post-smoothing starts from the prolongated coarse correction
        if constexpr (sizeof(T) == 4)
            init = post ? a.d1f : nullptr;
        else
            init = post ? a.d1 : nullptr;
        T *buf[2] = {e, scratch};
        T *out = buf[(steps - 1 - s) & 1];
        const T *prev = s > 0 ? buf[(steps - s) & 1] : init;
        bilu_step_body<T, TR, NT>(d.g, W, diag, shifted ? invd + d.g.N : invd, rhs, prev, out, w.blk, lds,
                                  block_shift(d.g, shifted), FromCoarse<T, void>{}, (int)threadIdx.x);
    }
}

// The batched FP32 step in the row form: work item = (instance, group of
// kRowBlocks blocks along x), kRowThreads threads per workgroup.
template <class T, class TR>
__global__ __launch_bounds__(kRowThreads) void kb_bilu_step_row(const InstDev *__restrict__ inst,
                                                                 const WorkItem *__restrict__ work,
                                                                 const int32_t *nwork, int post, int s, int steps)
{
    __shared__ SmoothLds<T> Ls[kRowBlocks];
    const int nw = *nwork;
    int t = blockIdx.x;
    WorkItem wnext = t < nw ? work[t] : WorkItem{0, 0};
    for (; t < nw; t += gridDim.x) {
        const WorkItem w = wnext;
        if (t + (int)gridDim.x < nw) wnext = work[t + gridDim.x];
        const InstDev &d = inst[w.inst];
        if (d.a.ictl[C_DONE]) continue;
        const Arrays &a = d.a;
        const int shifted = d.alt && (s & 1);
        T *buf[2] = {post ? a.d2f : a.d0f, a.zf};
        T *out = buf[(steps - 1 - s) & 1];
        const T *prev = s > 0 ? buf[(steps - s) & 1] : (post ? a.d1f : nullptr);
        const TR *rhs;
        if constexpr (sizeof(TR) == 4)
            rhs = a.r1f;
        else
            rhs = a.r;
        row_step_body<T, TR, kRowBlocks, kRowThreads>(d.g, a.W32, a.diag32, shifted ? a.invd32 + d.g.N : a.invd32,
                                                      rhs, prev, out, w.blk, Ls, block_shift(d.g, shifted),
                                                      (int)threadIdx.x);
    }
}

// Smoothing step on a grid with more blocks than are resident at once.
// FP32: four blocks along x per 512-thread workgroup (k_bilu_step_row: a
// wave's loads cover 128-byte rows); FP64: one 256-thread workgroup per
// block (the multi-block shapes measured slower there, see the design notes).
template <class T, class TR>
void launch_step_many(cams_ctx *c, const T *W, const T *diag, const T *iv, const TR *rhs, const T *prev, T *out,
                      const int32_t *done, int sh, int nb)
{
    if constexpr (sizeof(T) == 4) {
        constexpr int BPX = kRowBlocks, NT = kRowThreads;
        const GridDev &g = c->g;
        const int nbx = (g.nx + SB - 1) / SB, nby = (g.ny + SB - 1) / SB, nbz = (g.nz + SB - 1) / SB;
        const int wgs = ((nbx + BPX - 1) / BPX) * nby * nbz;
        if (wgs <= resident_workgroups((const void *)k_bilu_step_row<T, TR, BPX, NT>, NT))
            k_bilu_step_row<T, TR, BPX, NT><<<wgs, NT, 0, c->stream>>>(g, W, diag, iv, rhs, prev, out, done, sh);
        else
            k_bilu_step_rows<T, TR, BPX, NT><<<wgs, NT, 0, c->stream>>>(g, W, diag, iv, rhs, prev, out, done, sh);
    } else {
        k_bilu_step<T, TR, kSmoothThreadsMany, 0><<<nb, kSmoothThreadsMany, 0, c->stream>>>(c->g, W, diag, iv, rhs,
                                                                                            prev, out, done, sh);
    }
}

inline int num_sblocks(const GridDev &g)
{
    return ((g.nx + SB - 1) / SB) * ((g.ny + SB - 1) / SB) * ((g.nz + SB - 1) / SB);
}

}  // namespace

// Pivots of the block grid at the origin into invd[0, N); for the
// alternating smoother also those of the shifted grid into invd[N, 2N).
void launch_bilu_setup(cams_ctx *c)
{
    k_bilu_setup<<<num_sblocks(c->g), ST, 0, c->stream>>>(c->g, c->a.W, c->a.diag, c->a.invd, c->a.status, 0);
    if (c->opt.smoother == CAMS_SMOOTH_BLOCK_ALT_ILU0)
        k_bilu_setup<<<num_sblocks(c->g), ST, 0, c->stream>>>(c->g, c->a.W, c->a.diag, c->a.invd + c->g.N,
                                                             c->a.status, 1);
}

// Whether step s of a smoothing stage takes the shifted block grid.
static inline int step_shifted(const cams_ctx *c, int s)
{
    return c->opt.smoother == CAMS_SMOOTH_BLOCK_ALT_ILU0 && (s & 1);
}

template <class T, class TR>
void bilu_smooth(cams_ctx *c, const T *W, const T *diag, const T *invd, const TR *rhs, T *e, T *scratch, int steps,
                 const int32_t *done, const T *e_init)
{
    const int nb = num_sblocks(c->g);
    T *buf[2] = {e, scratch};
    const T *prev = e_init;
    // algorithmic bytes of a step: rhs, W (3), invd, e_new; plus diag and e_old after the first
    const double n = (double)c->g.N;
    double bytes = 0.0;
    for (int s = 0; s < steps; ++s)
        bytes += n * ((double)sizeof(TR) + 5.0 * sizeof(T) + (s > 0 || e_init ? 2.0 * sizeof(T) : 0.0));
    // the whole back-to-back sequence is bracketed, which keeps the event
    // overhead per launch small
    const bool timed = c->prof_kernel == CAMS_PROF_SMOOTH_STEP && c->prof_iter % kProfEvery == 0 && steps > 0;
    if (timed) prof_begin(c, bytes, steps);
    const bool in_regs = nb <= resident_workgroups((const void *)k_bilu_step<T, TR, kSmoothThreads, 1>, kSmoothThreads);
    for (int s = 0; s < steps; ++s) {
        T *out = buf[(steps - 1 - s) & 1];
        const int sh = step_shifted(c, s);
        const T *iv = sh ? invd + c->g.N : invd;
        if (in_regs)
            k_bilu_step<T, TR, kSmoothThreads, 1><<<nb, kSmoothThreads, 0, c->stream>>>(c->g, W, diag, iv, rhs,
                                                                                        prev, out, done, sh);
        else
            launch_step_many<T, TR>(c, W, diag, iv, rhs, prev, out, done, sh, nb);
        prev = out;
    }
    if (timed) prof_end(c);
}

// `steps` block-ILU(0) Richardson steps on A e = rhs from e = P xc (the
// prolongated coarse correction, Eq. (12)), the first with the prolongation
// inside it.  Timing (cams_profile) brackets the later steps, which are
// k_bilu_step launches.
template <class T, class TR, class TP>
void bilu_smooth_from_coarse(cams_ctx *c, const T *W, const T *diag, const T *invd, const TR *rhs, T *e, T *scratch,
                             int steps, const int32_t *done, const TP *P)
{
    if (steps <= 0) return;
    const int nb = num_sblocks(c->g);
    T *buf[2] = {e, scratch};
    const bool in_regs = nb <= resident_workgroups((const void *)k_bilu_first<T, TR, kSmoothThreads, 1, TP>,
                                                   kSmoothThreads);
    const double n = (double)c->g.N;
    const double bytes = (steps - 1) * n * ((double)sizeof(TR) + 7.0 * sizeof(T));
    const bool timed = c->prof_kernel == CAMS_PROF_SMOOTH_STEP && c->prof_iter % kProfEvery == 0 && steps > 1;
    T *out = buf[(steps - 1) & 1];
    if (in_regs)
        k_bilu_first<T, TR, kSmoothThreads, 1, TP><<<nb, kSmoothThreads, 0, c->stream>>>(
            c->g, W, diag, invd, rhs, P, c->a.dmask, c->a.xc, out, done);
    else
        k_bilu_first<T, TR, kSmoothThreadsMany, 0, TP><<<nb, kSmoothThreadsMany, 0, c->stream>>>(
            c->g, W, diag, invd, rhs, P, c->a.dmask, c->a.xc, out, done);
    const T *prev = out;
    if (timed) prof_begin(c, bytes, steps - 1);
    const bool regs_step = nb <= resident_workgroups((const void *)k_bilu_step<T, TR, kSmoothThreads, 1>,
                                                     kSmoothThreads);
    for (int s = 1; s < steps; ++s) {
        out = buf[(steps - 1 - s) & 1];
        const int sh = step_shifted(c, s);
        const T *iv = sh ? invd + c->g.N : invd;
        if (regs_step)
            k_bilu_step<T, TR, kSmoothThreads, 1><<<nb, kSmoothThreads, 0, c->stream>>>(c->g, W, diag, iv, rhs,
                                                                                        prev, out, done, sh);
        else
            launch_step_many<T, TR>(c, W, diag, iv, rhs, prev, out, done, sh, nb);
        prev = out;
    }
    if (timed) prof_end(c);
}

// Whether the first post-smoothing step takes the prolongation: when every
// block of the grid is resident at once (the launch is latency-bound and one
// launch less pays); on larger grids a separate prolongation is cheaper than
// prolongating each block's face neighbours again.
bool bilu_first_fused(cams_ctx *c)
{
    const int nb = num_sblocks(c->g);
    const void *k;
    if (c->opt.precision == CAMS_FP64)
        k = (const void *)k_bilu_first<double, double, kSmoothThreads, 1, double>;
    else if (c->opt.precision == CAMS_MIXED_BF16)
        k = (const void *)k_bilu_first<float, float, kSmoothThreads, 1, uint16_t>;
    else
        k = (const void *)k_bilu_first<float, float, kSmoothThreads, 1, float>;
    return nb <= resident_workgroups(k, kSmoothThreads);
}

void launch_bilu_smooth_from_coarse(cams_ctx *c, const double *rhs, double *e, int steps, const int32_t *done)
{
    bilu_smooth_from_coarse<double, double, double>(c, c->a.W, c->a.diag, c->a.invd, rhs, e, c->a.z, steps, done,
                                                    c->a.P);
}

void launch_bilu_smooth32_from_coarse(cams_ctx *c, const float *rhs, float *e, int steps, const int32_t *done)
{
    if (c->opt.precision == CAMS_MIXED_BF16)
        bilu_smooth_from_coarse<float, float, uint16_t>(c, c->a.W32, c->a.diag32, c->a.invd32, rhs, e, c->a.zf,
                                                        steps, done, c->a.Pbf);
    else
        bilu_smooth_from_coarse<float, float, float>(c, c->a.W32, c->a.diag32, c->a.invd32, rhs, e, c->a.zf, steps,
                                                     done, c->a.P32);
}

// e = result of `steps` block-ILU(0) Richardson steps on A e = rhs from e =
// e_init (0 when null).  Ping-pong between e and a scratch vector so the
// last step writes e; e_init must be neither.
void launch_bilu_smooth(cams_ctx *c, const double *rhs, double *e, int steps, const int32_t *done,
                        const double *e_init)
{
    bilu_smooth<double, double>(c, c->a.W, c->a.diag, c->a.invd, rhs, e, c->a.z, steps, done, e_init);
}

// The same in FP32 (mixed precision), on the rounded matrix and pivots.
void launch_bilu_smooth32(cams_ctx *c, const float *rhs, float *e, int steps, const int32_t *done,
                          const float *e_init)
{
    bilu_smooth<float, float>(c, c->a.W32, c->a.diag32, c->a.invd32, rhs, e, c->a.zf, steps, done, e_init);
}

void launch_bilu_smooth32(cams_ctx *c, const double *rhs, float *e, int steps, const int32_t *done,
                          const float *e_init)
{
    bilu_smooth<float, double>(c, c->a.W32, c->a.diag32, c->a.invd32, rhs, e, c->a.zf, steps, done, e_init);
}

template <class T, class TR>
void batch_smooth_nt(const BatchLaunch &L, int steps, int rhs_kind, int nt)
{
    for (int s = 0; s < steps; ++s) {
        if constexpr (sizeof(T) == 4)
            if (nt == 0) {   // row form (list of block groups)
                launch_persistent(kb_bilu_step_row<T, TR>, kRowThreads, L, L.inst, L.work, L.nwork, rhs_kind, s,
                                  steps);
                continue;
            }
        switch (nt) {
        case 128: launch_persistent(kb_bilu_step<T, TR, 128>, 128, L, L.inst, L.work, L.nwork, rhs_kind, s, steps); break;
        case 256: launch_persistent(kb_bilu_step<T, TR, 256>, 256, L, L.inst, L.work, L.nwork, rhs_kind, s, steps); break;
        default: launch_persistent(kb_bilu_step<T, TR, ST>, ST, L, L.inst, L.work, L.nwork, rhs_kind, s, steps); break;
        }
    }
}

// Batched smoothing for every instance, `steps` Richardson steps with `nt`
// threads per block (128, 256 or 512), or with nt = 0 (FP32 only) in the
// row form over the list of block groups.  rhs_kind 0: pre-smoothing on r from
// zero; 1: post-smoothing on r (its FP32 copy when mixed) from d1.
void launch_batch_smooth(const BatchLaunch &L, int steps, int rhs_kind, bool mixed, int nt)
{
    if (!mixed)
        batch_smooth_nt<double, double>(L, steps, rhs_kind, nt);
    else if (rhs_kind == 1)
        batch_smooth_nt<float, float>(L, steps, rhs_kind, nt);
    else
        batch_smooth_nt<float, double>(L, steps, rhs_kind, nt);
}

}  // namespace cams
