// Internal declarations of libcams: context, device grid descriptor and the
// host-side launchers of every kernel.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "cams.h"

namespace cams {

constexpr int kMaxRatio = 8;      // largest coarsening ratio the LDS local solves support
constexpr int kBlock = 256;       // threads per workgroup of the fine-grid kernels
constexpr int kBlockTriMin = 4096; // MSFE coarse grids above this many nodes use block-tridiagonal elimination
constexpr int kStagWindow = 100;   // C-AMS iterations without a kStagDrop reduction of ||r|| = stagnation
constexpr double kStagDrop = 0.9;

// Grid descriptor passed by value to kernels.  Per-axis tables live in the
// workspace: vertex coordinates (nb entries), "is vertex coordinate" flags
// and the lower bracketing vertex of every coordinate (n entries).
// Row form of the residual-restriction: a workgroup takes up to kRowBoxes
// consecutive boxes along x whose cells fit rows of kRowCells.
constexpr int kRowCells = 32;
// Coarse sizes up to which every coarse-GEMV workgroup forms R r itself;
// larger dense MSFE inverses take the symmetric tile GEMV.
constexpr int kGemvLds = 1024;
constexpr int kRowBoxes = 8;

struct GridDev {
    int nx, ny, nz, N, sxy;
    double dx, dy, dz, dV;
    int nb[3];
    int r[3];
    int Nc;
    int dim;
    const int32_t *vc[3];
    const int32_t *lo[3];
    const uint8_t *isv[3];
    const int32_t *ob[3];   // restriction-owner box starts per axis (nb + 1 entries)
    // Groups of consecutive boxes along x whose cells fit a 32-cell row, for
    // the residual-restriction: gx[v] holds the first box of each group
    // (ngx[v] + 1 entries) over the primal blocks (v = 0) or the owner boxes
    // of the table ob (v = 1).
    const int32_t *gx[2];
    int ngx[2];
};

struct Fluid {
    double rho0, c, p0, mu, dt;
};

// Dirichlet boundary faces (fixed pressure on the west face x = 0 and / or
// the east face x = nx - 1), passed by value to the residual kernels.
struct FaceBC {
    double p[2];
    int on[2];
};

// One dual region (edge segment, face patch or interior box): per axis the
// first cell and the number of cells; `nfree` axes are open intervals.
struct Region {
    int32_t s[3];
    int32_t len[3];
    int32_t freemask;   // bit a set: axis a is an open interval
    int32_t pad;
};

// Pointers into the caller's workspace.
struct Arrays {
    double *T;        // 3N: Tx, Ty, Tz
    double *phi, *q;  // N, N (q only when sources are given)
    double *W;        // 3N: masked off-diagonal magnitudes of A
    double *diag, *r0, *r;
    double *dp[2];    // ping-pong accumulated update
    double *d0, *d1, *d2, *z, *x, *invd;
    double *P;        // 8N slot-major
    double *Ac, *Ainv, *work; // Nc*Nc each
    double *rc, *xc;  // Nc
    double *partial;  // reduction partials
    double *slots;    // Nc*8 restriction partials: slot s of owner box k
    double *boxp;     // Nc*216 coarse-operator partials of the owner boxes (MSFE)
    void *gjd;        // GEMM descriptors of the Gauss-Jordan inverse (MSFE)
    double *gjcb;     // Gauss-Jordan sweep buffers: old column blocks, their transposes, G (5 x 64 x matrix order per chain)
    double *scal;     // device scalars
    int32_t *piv;     // Nc
    int32_t *status;  // device error flags
    int32_t *ictl;    // iteration control: [0] iteration, [1] done, [2] outcome, [3] arrival counter,
                      // [4..4+Nc) per-node arrival counters of the restriction
    uint8_t *dmask;   // N
    int32_t *wcell;   // wells
    double *wp;
    int32_t *tab;     // per-axis tables
    Region *regions;  // dual regions of all stages
    // basis types B1-B3: couplings and extra diagonal of the local problems,
    // their snapshot at each region's last solve, per-region change flags and
    // the list of regions to re-solve (B1/B2 adaptive updates)
    double *bcoef, *bdiag, *bsnap, *bdsnap;
    double *Tb;       // 2 ny nz: half-cell transmissibilities of the west and east boundary faces
    double *Acs;      // 27 Nc: the coarse operator's 27-point entries when it was last factorised
    double *gpart;    // T^2 x 64 (T = ceil(Nc / 64)): tile partials of the symmetric coarse GEMV
    float *Ainv32;    // Nc*Nc: the lower-triangle tiles of Ainv rounded to FP32 (mixed precision, symmetric GEMV)
    int32_t *rflag;
    Region *rlist;
    // mixed precision copies
    float *W32, *diag32, *invd32, *P32;
    uint16_t *Pbf;
    float *r1f, *d0f, *d1f, *d2f, *zf;
};

// One instance of a batched solve as the batched kernels see it (a copy of
// its context's grid descriptor and workspace pointers).
struct InstDev {
    GridDev g;
    Arrays a;
    int fe;           // MSFE restriction
    int bf16;         // mixed precision with a bfloat16 basis
    int n_pre, n_post;
    int alt;          // alternating block smoother (odd steps on the shifted block grid)
    int nparts;       // residual partials: Nc (fused residual-restriction) or ceil(N / kBlock)
    int maxit;
    double rtol2;
};

// The share of a batched launch given to one workgroup.
struct WorkItem {
    int32_t inst;     // instance
    int32_t blk;      // block of that instance (meaning set by the kernel)
};

// A batched launch: `grid` persistent workgroups take the work items
// blockIdx.x, blockIdx.x + grid, ... below the device-side count *nwork (the
// list shrinks between launches as instances stop).
struct BatchLaunch {
    const InstDev *inst;
    const WorkItem *work;
    const int32_t *nwork;
    int grid;
    hipStream_t stream;
};

// Workgroups of `kernel` (with `threads` per workgroup) that the device
// holds at once: occupancy per CU x number of CUs, queried once per kernel.
int resident_workgroups(const void *kernel, int threads);

// Launch a persistent batched kernel with as many workgroups as are resident
// at once, at most L.grid (the list's full length).  With L.grid == 0 it
// launches nothing but still caches the occupancy (done before any graph
// capture, so that capture records launches only).
template <class K, class... Args>
inline void launch_persistent(K kernel, int threads, const BatchLaunch &L, Args... args)
{
    const int res = resident_workgroups((const void *)kernel, threads);
    if (L.grid <= 0) return;
    const int grid = L.grid < res ? L.grid : res;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), 0, L.stream, args...);
}

// Per-instance results copied to the host after a batched solve.
struct BatchResult {
    int32_t it, done, outcome, status;
    double eps2, r0n2, rn2;
};

// Slots of Arrays::ictl (iteration control).
enum { C_IT = 0, C_DONE = 1, C_OUTCOME = 2, C_ARRIVE = 3, C_NODE = 4 };

// Scalar slots in Arrays::scal.
enum { S_EPS2 = 0, S_R0N2 = 1, S_RN2 = 2, S_ATOL2 = 3, S_EPSH = 4, S_CCHG = 5 };

// Device status flags (bitwise OR).
enum { F_BAD_PIVOT = 1, F_BAD_INPUT = 2, F_SINGULAR_COARSE = 4 };

}  // namespace cams

// Norm histories of cams_newton_history: one entry per evaluated C-AMS
// residual (Newton index, ||r||_2, ||eps||_2 at the current iterate).
struct cams_history {
    double *res, *err;
    int32_t *newton;
    int cap, count, nu;
    const double *p, *pn;   // Newton iterate and old-time pressure of the running solve
};

struct cams_ctx {
    cams_grid grid;
    cams_fluid fluid;
    cams_options opt;
    hipStream_t stream;
    cams::GridDev g;
    cams::Fluid fl;
    int nreg[4];            // regions per stage (index = number of free axes)
    int regoff[4];
    int region_total;
    int maxm[4], maxbw[4];  // largest local system per stage
    int nfull;              // interior regions that are full 7x7x7 dual blocks (listed first)
    bool blocktri;          // coarse operator factorised by block-tridiagonal elimination over z-planes
    // learned basis: network parameters and scratch (caller-owned), settings, counters
    const float *learned_params;
    char *learned_scratch;
    size_t learned_scratch_bytes;
    double fallback_tol;
    int guard_iters;          // exact-basis iterations per solve for the global check (0: off)
    bool learned_suspended;   // the global check switched the basis to local solves
    int learned_blocks, fallback_blocks;
    std::vector<cams::Region> fallback_list;
    std::vector<double> block_ratio;   // local-equation ratio of each full block in the last learned build
    size_t need;
    char *ws;
    size_t ws_bytes;
    cams::Arrays a;
    int nparts;             // reduction partial count
    int nwells;
    bool has_ws, has_rock, has_q, has_basis, has_system, has_coarse;
    bool ac_zeroed;         // A_c outside the 27-point pattern zeroed in this workspace
    bool gj_ready;          // Gauss-Jordan descriptors uploaded for this workspace
    std::vector<int> gj_launch;   // per GEMM launch of the inverse: offset, count, tiles
    int cur_dp;
    double *host;           // pinned host scalars
    hipEvent_t ev[8];
    // second stream and its fork / join events (block-tridiagonal factorisation only)
    hipStream_t side;
    hipEvent_t fork_ev, join_ev;
    cams_stats last;
    cams_history *hist;     // non-null while cams_newton_history runs
    std::string err;
    // host copies of the per-axis tables and dual regions (uploaded by
    // cams_set_workspace) and the workspace offsets
    std::vector<int32_t> tab;
    std::vector<cams::Region> regions;
    size_t tab_off[3][4];
    size_t tab_gx[2];
    // the pair form of the residual-restriction applies (nx and every box
    // edge along x even), per restriction type as tab_gx
    bool row_pairs[2];
    // timing of one kernel class for measurement (cams_profile)
    int prof_kernel;
    std::vector<hipEvent_t> prof_ev;        // pool: pairs (start, stop)
    std::vector<int> prof_tag;              // iteration index of each pair
    std::vector<double> prof_bytes_pair;    // algorithmic bytes of each pair
    std::vector<int> prof_count_pair;       // kernel launches inside each pair
    int prof_used;
    int prof_iter;                          // iteration index being enqueued
    double prof_ms, prof_bytes;
    long long prof_launches;
    size_t off[64];         // workspace offsets (kMaxArrays entries)
    // pressure-dependent bases (B1/B2): coefficients assembled for the current
    // iterate, and for each region the regions that take its values as
    // boundary data (CSR over the region order of `regions`)
    bool has_bcoef;
    cams::FaceBC bc;        // Dirichlet boundary faces (cams_set_face_dirichlet)
    bool has_cfac;          // Ainv holds a factorisation of the operator snapshotted in Acs
    bool ainv32_ok;         // Ainv32 holds the current Ainv rounded (false after a batched factorisation)
    int n_factor;           // coarse factorisations since the last reset of the counter
    std::vector<int32_t> dep_ptr, dep_idx;
};

namespace cams {

// ---- fine-grid kernels (k_fine.hip)
void launch_fill(cams_ctx *c, double *x, int n, double v);
void launch_transmissibility(cams_ctx *c, const double *perm);
void launch_check_rock(cams_ctx *c, const double *perm, const double *phi);
void launch_assemble(cams_ctx *c, const double *p, const double *pn);
void launch_reduce(cams_ctx *c, const double *partial, int n, double *out);
// ||eps||^2 (Eq. (16)) at x = p + dp (dp nullable) into *out, without
// touching the assembled system; partials in Arrays::partial.
void launch_eps_at(cams_ctx *c, const double *p, const double *dp, const double *pn, double *out);
// Basis types B1-B3 (Sec. 3): local-problem coefficients at the iterate p
// (B1/B2) or from the rock (B3); per-region coefficient change against the
// snapshot (flags of regions [first, first + count)); snapshot of listed regions.
void launch_basis_coeffs(cams_ctx *c, const double *p, const double *pn);
void launch_region_change(cams_ctx *c, int first, int count, double tol);
void launch_region_snapshot(cams_ctx *c, const Region *regs, int count);
// Two-point mass fluxes (3N, on the lower cell of each face) of the system
// assembled at p, at the pressure p + d.
void launch_face_flux(cams_ctx *c, const double *p, const double *d, double *flux);
// Zero the coarse operator once per workspace (entries outside the 27-point
// pattern stay zero afterwards).
void launch_zero_coarse(cams_ctx *c);
// Largest relative change of the coarse operator's 27-point entries since
// the snapshot (into scal[S_CCHG]), or (snap) take the snapshot.
void launch_coarse_change(cams_ctx *c, bool snap);
void launch_impose_wells(cams_ctx *c, double *p);
void launch_stencil_sub(cams_ctx *c, const double *b, const double *x, double *out, const int32_t *done);
void launch_prolong(cams_ctx *c, const double *xc, double *out, const int32_t *done);
void launch_ilu_setup(cams_ctx *c);  // dispatches on opt.smoother
void launch_rb_setup(cams_ctx *c);
void launch_rb_smooth(cams_ctx *c, const double *rhs, double *e, int steps);
void launch_nat_setup(cams_ctx *c);
void launch_nat_smooth(cams_ctx *c, const double *rhs, double *e, int steps);
// Block ILU(0) smoothers (BLOCK, BLOCK_ALT): the forms with device stop
// flags, mixed-precision variants and batched kernels.
inline bool block_smoother(const cams_options &o)
{
    return o.smoother == CAMS_SMOOTH_BLOCK_ILU0 || o.smoother == CAMS_SMOOTH_BLOCK_ALT_ILU0;
}
// dispatches on opt.smoother; `done` (nullable) skips the work once the iteration has converged
void launch_smooth(cams_ctx *c, const double *rhs, double *e, int steps, const int32_t *done);
void launch_axpy(cams_ctx *c, double *y, const double *x, int n);

// ---- block ILU(0) smoother (k_smooth.hip)
void launch_bilu_setup(cams_ctx *c);
void launch_bilu_smooth(cams_ctx *c, const double *rhs, double *e, int steps, const int32_t *done,
                        const double *e_init = nullptr);

// post-smoothing from e = P xc, the prolongation fused into the first step
// (when bilu_first_fused: grids whose blocks are all resident at once)
bool bilu_first_fused(cams_ctx *c);
void launch_bilu_smooth_from_coarse(cams_ctx *c, const double *rhs, double *e, int steps, const int32_t *done);
void launch_bilu_smooth32_from_coarse(cams_ctx *c, const float *rhs, float *e, int steps, const int32_t *done);
void launch_bilu_smooth32(cams_ctx *c, const float *rhs, float *e, int steps, const int32_t *done,
                          const float *e_init = nullptr);
void launch_bilu_smooth32(cams_ctx *c, const double *rhs, float *e, int steps, const int32_t *done,
                          const float *e_init = nullptr);

// measurement hooks around the smoothing-step launches (abi.hip); only the
// launches of every kProfEvery-th iteration are bracketed by events, which
// keeps the event overhead out of the rest of the timed run
constexpr int kProfEvery = 16;
void prof_begin(cams_ctx *c, double bytes, int launches);
void prof_end(cams_ctx *c);

// ---- mixed precision (k_mixed.hip)
void launch_convert_matrix32(cams_ctx *c);   // W, diag, invd -> FP32 copies
void launch_round_basis(cams_ctx *c);        // P -> FP32 / BF16, P := the rounded values
void launch_prolong32(cams_ctx *c, const double *xc, float *out, const int32_t *done);
void launch_sub64_lo(cams_ctx *c, const float *x, double *r, const int32_t *done);   // and r1f = (float) r

// ---- iteration control (k_iter.hip)
void launch_iter_reset(cams_ctx *c);
// r = r0 - A v with v = dp_in (+ the pending corrections after the first
// iteration), dp_out = v, ||r|| and the stopping test on the device
void launch_residual_ctl(cams_ctx *c, const double *dp_in, const double *a0, const double *a1, const double *a2,
                         double *dp_out);
void launch_residual_ctl32(cams_ctx *c, const double *dp_in, const float *a0, const float *a1, const float *a2,
                           double *dp_out, float *rf);   // also rf = (float) r
// residual and restriction slots in one pass (no pre-smoothing); partial[k] per owner box
void launch_residual_restrict(cams_ctx *c, const double *dp_in, const double *a0, const double *a1,
                              const double *a2, double *dp_out);
void launch_residual_restrict32(cams_ctx *c, const double *dp_in, const float *a0, const float *a1, const float *a2,
                                double *dp_out, float *rf);
void launch_finalize_ctl(cams_ctx *c, int nparts);   // ||r|| from nparts partials, stopping test, counter
void launch_restrict(cams_ctx *c, const double *r);   // slot partials of R r (stage 1)

// ---- setup phases without host synchronisation (abi.hip)
void enqueue_clear_status(cams_ctx *c);
void enqueue_assemble(cams_ctx *c, const double *p, const double *pn);
void enqueue_basis_local(cams_ctx *c);
void enqueue_coarse_operator(cams_ctx *c);   // A_c, smoother pivots, FP32 copies (no factorisation)
void enqueue_coarse(cams_ctx *c);

// ---- batched iteration (one launch per kernel for all instances)
void launch_batch_residual(const BatchLaunch &L, int par, bool mixed, bool pre);
void launch_batch_finalize(const InstDev *inst, int count, hipStream_t st);
void launch_batch_restrict(const BatchLaunch &L, int precision);
void launch_batch_gather(const InstDev *inst, int count, BatchResult *out, hipStream_t st);
void launch_batch_reset(const BatchLaunch &L);   // iteration state of every instance to its start
void launch_batch_node_sum(const BatchLaunch &L);
void launch_batch_gemv(const BatchLaunch &L);
void launch_batch_prolong(const BatchLaunch &L, bool mixed, bool bf16);
void launch_batch_sub_pre(const BatchLaunch &L, bool mixed);
void launch_batch_smooth(const BatchLaunch &L, int steps, int rhs_kind, bool mixed, int nt);
void launch_batch_update(const BatchLaunch &L, double *const *p);
void launch_batch_prolong64(const BatchLaunch &L);
void launch_batch_sub_pre64(const BatchLaunch &L);

// ---- basis (k_basis.hip)
void launch_basis(cams_ctx *c);
void launch_basis_vertices(cams_ctx *c);
void launch_basis_regions(cams_ctx *c, int nfree, const Region *regs, int count);
void launch_batch_basis_regions(const InstDev *inst, const WorkItem *items, int count, int nfree, int cap,
                                hipStream_t st);

// ---- learned basis network (k_cnn.hip)
size_t cnn_num_params();
size_t cnn_workspace_floats(int B);
void cnn_forward(hipStream_t st, const float *params, const float *feat, int B, float *ws, float *phi_out);
void cnn_loss_grad(hipStream_t st, const float *params, const float *feat, const float *target, int B, float *ws,
                   float *grad, double *loss_out);
void cnn_adam(hipStream_t st, float *p, const float *g, float *m, float *v, int n, int t, float lr, float b1,
              float b2, float eps);
size_t cnn_bf16_bytes();
void cnn_forward_bf16(hipStream_t st, const float *params, const float *feat, int B, void *wb, float *phi_out);
void cnn_features(cams_ctx *c, const Region *regs, int nblk, float *feat);
void cnn_targets(cams_ctx *c, const Region *regs, int nblk, float *tgt);
void cnn_scatter(cams_ctx *c, const Region *regs, int nblk, const float *phi);
void cnn_block_residual(cams_ctx *c, const Region *regs, int nblk, double *ratio);

// ---- batched coarse factorisation (k_coarse.hip)
// One Gauss-Jordan pivot step of one instance: the inverse of the nb x nb
// pivot block of A (n x n) at (j0, j0) and the copy of its old column block
// into Cb; its workgroups are wg0 .. wg0 + 1 + ceil((n - nb) nb / 256) - 1
// of the launch.
struct GjPivotDesc {
    double *A, *Cb, *CbT;
    int32_t *status;
    int n, j0, nb, wg0;
};
// C = alpha A B + beta C for one instance; its tiles are tile0 .. tile0 +
// tiles_n * ceil(M / 64) - 1 of the launch.
struct GemmDesc {
    double *C;
    const double *A, *B;
    int ldc, lda, ldb, M, N, K;
    double alpha, beta;
    int tiles_n, tile0;
    // Optional (null when unused; k_gj_panel_sym only): the A operand is not
    // read from memory but formed per tile as the tile's rows of S (row
    // pitch lda) times pre (K x K, row pitch ldc).
    const double *pre, *S;
    // tri: the tiles are those of the lower triangle (diagonal tiles whole)
    // of the square M x N region, counted row by row.
    int tri;
};
struct BatchGjPlan {
    enum Kind { PIVOT = 0, PANEL = 1, UPDATE_PIVOT = 2, MIRROR = 3 };
    struct Launch {
        int kind;
        size_t poff;    // into piv
        int pcount, pw; // pivot descriptors and their workgroups
        size_t goff;    // into gemms
        int gcount, tiles;
    };
    std::vector<GjPivotDesc> piv;
    std::vector<GemmDesc> gemms;
    std::vector<Launch> launches;
};
void launch_coarse_factor_prepare(cams_ctx *c);
void plan_batch_gj(const std::vector<cams_ctx *> &fe, BatchGjPlan &plan);
void launch_batch_gj(const BatchGjPlan &plan, const GjPivotDesc *piv, const GemmDesc *gemms, hipStream_t st);

// ---- coarse level (k_coarse.hip)
void launch_coarse_operator(cams_ctx *c);
void launch_coarse_factor(cams_ctx *c);   // LU + explicit inverse of Ac
void launch_gemv(cams_ctx *c, const double *rc, double *xc, const int32_t *done, int stop_parts = 0);
void launch_coarse_solve(cams_ctx *c, const double *rc, double *xc);   // xc = A_c^-1 rc

}  // namespace cams

#define CAMS_HIP(call)                                                   \
    do {                                                                 \
        hipError_t e_ = (call);                                          \
        if (e_ != hipSuccess) throw cams::HipError(e_, #call, __LINE__); \
    } while (0)

namespace cams {
struct HipError {
    hipError_t code;
    const char *what;
    int line;
    HipError(hipError_t c, const char *w, int l) : code(c), what(w), line(l) {}
};
}  // namespace cams
