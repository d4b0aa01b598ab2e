/*
 * cams.h — C ABI of the MI355X C-AMS pressure solver (libcams.so).
 *
 * Compressible algebraic multiscale solver (C-AMS) of Tene, Wang and
 * Hajibeygi, "Adaptive Algebraic Multiscale Solver for Compressible Flow in
 * Heterogeneous Porous Media" (arXiv 1705.05783).  Equations are numbered in
 * order of appearance in the paper: (1) mass balance, (2) backward-Euler
 * nonlinear pressure equation, (3)-(5) its linearisation, (6) the algebraic
 * system, (7) finite-volume restriction, (8)-(11) basis types B1-B4, (12)
 * superposition, (13) coarse system R A P, (14)-(15) multiscale solution and
 * correction, (16) nonlinear error.  Table "cams" is the iteration procedure.
 *
 * Conventions shared by every entry point
 *  - Cells are indexed n = i + nx*(j + ny*k), x fastest, zero based.  A grid
 *    with nz == 1 is two-dimensional.
 *  - Every array argument named *_dev is DEVICE memory on the context's
 *    device, FP64 unless stated, borrowed for the duration of the call only
 *    (the library keeps no pointer to it).  Arrays named *_host are host
 *    memory, copied before the call returns.
 *  - All device work is enqueued on the HIP stream given to cams_create.
 *    Calls that return a host-visible number (eps_norm_out, cams_stats)
 *    synchronise that stream; the others return after enqueueing.  The one
 *    exception is the block elimination of cams_coarse_op (below): half of
 *    it runs on a second stream that the context creates (default priority)
 *    and joins back to the given stream with an event before the call
 *    returns, so later work on the given stream sees the complete result.
 *  - The library allocates no device memory of its own beyond one small
 *    pinned host buffer: all device state lives in a caller-provided
 *    workspace (cams_workspace_bytes / cams_set_workspace), typically a
 *    torch.empty(..., dtype=torch.uint8) buffer.  The workspace must outlive
 *    the context.
 *  - Errors are returned as cams_status; nothing is thrown across the ABI.
 *    cams_last_error gives a readable message for the last failure.
 *  - A context is not thread safe; distinct contexts are independent.
 */
#ifndef CAMS_H
#define CAMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cams_ctx cams_ctx;

typedef enum {
    CAMS_OK = 0,
    CAMS_E_ARG = -1,           /* invalid argument (checked on the host before any device work) */
    CAMS_E_STATE = -2,         /* call out of order (e.g. iterate before assemble) */
    CAMS_E_DEVICE = -3,        /* a HIP runtime call failed */
    CAMS_E_NOMEM = -4,         /* workspace missing or too small */
    CAMS_E_NOT_CONVERGED = -5, /* iteration limit reached; last iterate is kept */
    CAMS_E_BREAKDOWN = -6      /* NaN/Inf norm, zero pivot or non-positive local pivot */
} cams_status;

/* Restriction operator (Sec. 3): finite volume, Eq. (7), or finite element R = P^T. */
enum { CAMS_R_FV = 0, CAMS_R_FE = 1 };

/* Arithmetic of the solve.  FP64: everything in double.  MIXED_FP32: a float
 * copy of the matrix and smoother pivots, the smoother, the basis storage and
 * the prolongation in float with float accumulation; residual, Newton
 * update, norms, coarse operator and coarse solve in double (iterative
 * refinement on the FP64 residual).  The basis is computed in double and
 * rounded once; the coarse operator and the restriction use the rounded
 * basis.  MIXED_BF16: as MIXED_FP32 but the basis stored in bfloat16. */
enum { CAMS_FP64 = 0, CAMS_MIXED_FP32 = 1, CAMS_MIXED_BF16 = 2 };

/* ILU(0) smoother of Table "cams" step 6.  BLOCK: block-Jacobi ILU(0) in
 * natural order on 8x8x8 cell blocks aligned at the origin (8x8 in 2D; the
 * last block of an axis may be shorter), couplings across block faces left
 * out of the factor only.  RB: ILU(0) of the whole matrix in red-black
 * order (even i+j+k first).  BLOCK_ALT: the Richardson steps of each
 * smoothing stage alternate between the BLOCK factor and block-Jacobi
 * ILU(0) on the block grid shifted cyclically by half a block on every
 * axis longer than one block (cell i at position (i + 4) mod nx along x,
 * blocks of 8 consecutive positions; likewise y and z; an axis of at most 8
 * cells is one block either way); the first step of a stage takes the grid
 * at the origin.  A closer stand-in for the paper's global ILU(0):
 * fewer iterations for the same work per step.  NAT: ILU(0) of the whole
 * matrix in natural (cell) order, the paper's own smoother; its triangular
 * solves are wavefronts over the grid's diagonals (one launch per diagonal
 * of 16 x 16 x 8 cell bricks), so a step costs far more than a block step
 * and the iteration count is the reference the block forms are judged by.
 * RB and NAT are FP64 only and take no part in batches. */
enum { CAMS_SMOOTH_BLOCK_ILU0 = 0, CAMS_SMOOTH_RB_ILU0 = 1, CAMS_SMOOTH_BLOCK_ALT_ILU0 = 2,
       CAMS_SMOOTH_NAT_ILU0 = 3 };

/* Basis function type (Sec. 3, Eqs. (8)-(11)), each solved with the same
 * reduced-problem boundary conditions, in the mass form of the Newton
 * system (rows multiplied by rho dV):
 *   B4 (default): -div(lambda grad Phi) = 0: couplings T; pressure
 *       independent, built once per rock;
 *   B3: c^n Phi - div(lambda grad Phi) = 0: couplings T plus the diagonal
 *       phi c dV / dt (c^n at the old time level; pressure independent);
 *   B2: -(1/rho) div(rho lambda grad Phi) = 0: couplings
 *       T (rho_i + rho_j)/2 of the current Newton iterate;
 *   B1: c Phi - (1/rho) div(rho lambda grad Phi) = 0: those couplings plus
 *       the accumulation diagonal of the Newton matrix, phi c rho(p^n) dV/dt.
 * B1 and B2 depend on pressure: cams_newton_step updates them adaptively at
 * every Newton iteration (see basis_tol).  With an accumulation term (B1,
 * B3) the basis is not a partition of unity. */
enum { CAMS_BASIS_B4 = 0, CAMS_BASIS_B1 = 1, CAMS_BASIS_B2 = 2, CAMS_BASIS_B3 = 3 };

typedef struct {
    int32_t nx, ny, nz;       /* fine cells per axis, >= 2 on active axes (nz == 1 for 2D) */
    double dx, dy, dz;        /* cell sizes (> 0) */
    int32_t rx, ry, rz;       /* coarsening ratio per axis, 2..8 (rz = 1 in 2D) */
} cams_grid;

/* Fluid and time step (Sec. 2, Eqs. (1)-(2)): rho(p) = rho0 exp(c (p - p0)),
 * viscosity mu, backward-Euler step dt. */
typedef struct {
    double rho0, c, p0, mu, dt;
} cams_fluid;

typedef struct {
    int32_t restriction;      /* CAMS_R_FV or CAMS_R_FE */
    int32_t n_pre;            /* ILU(0) Richardson steps before the multiscale stage (0..64) */
    int32_t n_post;           /* ILU(0) Richardson steps after it (Table "cams" step 6; 0..64) */
    int32_t precision;        /* CAMS_FP64 / CAMS_MIXED_FP32 / CAMS_MIXED_BF16 */
    int32_t smoother;         /* CAMS_SMOOTH_BLOCK_ILU0, _RB_ILU0, _BLOCK_ALT_ILU0 or _NAT_ILU0 */
    double lin_rtol;          /* stop when ||r||_2 <= lin_rtol ||r0||_2 */
    int32_t lin_maxit;        /* linear iteration limit */
    double newton_tol;        /* stop Newton when ||eps||_2 <= newton_tol (Eq. (16)) */
    int32_t newton_maxit;     /* Newton iteration limit per time step */
    double lin_atol;          /* also stop when ||r||_2 <= lin_atol (absolute; 0 = relative test only) */
    int32_t basis_type;       /* CAMS_BASIS_B4 (0, default), B1, B2 or B3 */
    double basis_tol;         /* B1/B2 adaptive update: a dual region is re-solved when a coefficient of
                                 its local problem changed by more than this (relative) since it was
                                 last solved, and so is every region that takes it as boundary data;
                                 0 = every region at every Newton iteration */
    double coarse_tol;        /* adaptive coarse factorisation: cams_coarse_op keeps the last inverse
                                 while no entry of R A P_hat changed by more than this (relative) since
                                 it was factorised; 0 (default) = factorise at every call, as Table
                                 "cams" updates the system at every Newton iteration */
} cams_options;

typedef struct {
    int32_t newton_iters;     /* linear solves performed in the last cams_newton_step */
    int32_t lin_iters_total;  /* C-AMS iterations summed over those solves */
    int32_t lin_iters_last;   /* C-AMS iterations of the last cams_iterate */
    int32_t fallback_blocks;  /* learned basis: blocks re-solved exactly in the basis build (0 otherwise) */
    double relres_last;       /* ||r||/||r0|| at the end of the last cams_iterate */
    double eps_norm_last;     /* last ||eps||_2 from cams_assemble */
    double t_assemble_ms;     /* device time of the last newton step's phases (hipEvent) */
    double t_basis_ms;
    double t_coarse_ms;
    double t_iterate_ms;
    int32_t basis_updates;          /* B1/B2: adaptive basis updates in the last cams_newton_step */
    int32_t basis_regions_rebuilt;  /* dual regions solved by the basis builds and updates of that step */
    int32_t coarse_factorizations;  /* coarse inverses computed in that step (< newton_iters with coarse_tol) */
    int32_t basis_rebuilds;         /* learned basis replaced by local solves in that step (the check of
                                     * cams_set_learned_guard; 0 or 1) */
} cams_stats;

/* Create a context for one grid.  Validates grid/fluid/options: active axes
 * >= 2 cells, 2 <= r <= 8 and r <= n per axis, vertex spacing >= 2 cells,
 * at most 32768 coarse nodes, dx,dy,dz,dt,mu,rho0 > 0, c >= 0, tolerances
 * > 0; the mixed precisions need a block smoother (BLOCK or BLOCK_ALT).  `hip_stream` is a
 * hipStream_t (NULL = default
 * stream).  Makes no HIP call (works without a GPU); on success *out owns
 * no device memory.  Release with cams_destroy.  Errors: CAMS_E_ARG,
 * CAMS_E_NOMEM (host allocation). */
cams_status cams_create(const cams_grid *grid, const cams_fluid *fluid, const cams_options *opt,
                        void *hip_stream, cams_ctx **out);

/* Bytes of device workspace the context needs (256-byte aligned). */
size_t cams_workspace_bytes(const cams_ctx *ctx);

/* Hand over the device workspace: `dev_ptr` must be 256-byte aligned and hold
 * at least cams_workspace_bytes() bytes; its contents are overwritten and
 * all rock, well and basis state is reset.  The first call also allocates a
 * 4 KB pinned host buffer for scalar read-backs.
 * Errors: CAMS_E_ARG (null, misaligned), CAMS_E_NOMEM (too small),
 * CAMS_E_DEVICE. */
cams_status cams_set_workspace(cams_ctx *ctx, void *dev_ptr, size_t bytes);

/* Rock properties (Sec. 2): isotropic permeability perm_dev[N] (> 0), porosity
 * phi_dev[N] (0 < phi <= 1), optional source q_dev[N] per unit volume (NULL =
 * none).  Copies them into the workspace and computes the two-point
 * transmissibilities (harmonic average of the two half-cell conductances,
 * Eq. (6)).  Invalidates any basis already built.
 * Errors: CAMS_E_STATE (no workspace), CAMS_E_ARG (null pointers, or a
 * permeability or porosity value out of range: checked on the device, so
 * this call synchronises the stream). */
cams_status cams_set_rock(cams_ctx *ctx, const double *perm_dev, const double *phi_dev,
                          const double *q_dev);

/* Mark the basis (and the coarse operator) stale, so that the next
 * cams_newton_step or batched iteration rebuilds it from the current
 * transmissibilities.  Host only; no device call. */
cams_status cams_invalidate_basis(cams_ctx *ctx);

/* Dirichlet (well) cells: cells_host[n] are cell indices, p_host[n] their fixed
 * pressures (wells as fixed-pressure cells, Sec. 4.2 test case 2).
 * Replaces any earlier set.  n = 0 removes all wells (then c > 0 is required
 * for a non-singular system).  Errors: CAMS_E_ARG (index out of range,
 * duplicate, non-finite pressure), CAMS_E_STATE (no workspace). */
cams_status cams_set_wells(cams_ctx *ctx, const int64_t *cells_host, const double *p_host, int32_t n);

/* Dirichlet boundary face (Sec. 4: the default test cases fix the pressure
 * on the west and east faces, no flow elsewhere): face 0 = west (x = 0),
 * 1 = east (x = nx - 1), at `pressure`; NaN removes it.  Every cell on that
 * face gets the two-point flux T_b (rho_i + rho(p_b))/2 (p_i - p_b) through
 * it, with T_b = 2 (k_i / mu) dy dz / dx the half-cell transmissibility
 * between the cell centre and the face, in the residual and (with the face
 * density frozen, as for interior faces) on the diagonal of the Newton
 * matrix.  The basis (Eq. (11)) is unaffected.  Host only; call before
 * cams_set_wells when the faces are the only Dirichlet data with c = 0.
 * Errors: CAMS_E_ARG (face, infinite pressure). */
cams_status cams_set_face_dirichlet(cams_ctx *ctx, int32_t face, double pressure);

/* Assemble the Newton linear system at pressure p_dev, old-time pressure
 * pn_dev (Sec. 2, Eqs. (2)-(6), multiplied by rho_i dV_i):
 *   A_ii = phi_i c rho(pn_i) dV/dt + sum_j W_ij,  A_ij = -W_ij,
 *   W_ij = T_ij (rho(p_i) + rho(p_j))/2,  r = -F(p)
 * with Dirichlet rows/columns set to identity and r = 0 there.  Writes the
 * nonlinear error norm ||eps||_2 (Eq. (16), eps_i = F_i/(rho_i dV)) to
 * *eps_norm_out (host pointer, may be NULL; non-NULL synchronises).
 * Errors: CAMS_E_STATE (no rock), CAMS_E_ARG, CAMS_E_DEVICE. */
cams_status cams_assemble(cams_ctx *ctx, const double *p_dev, const double *pn_dev,
                          double *eps_norm_out);

/* Build the prolongation from basis type B4 (Sec. 3, Eq. (11)) with
 * reduced-problem boundary conditions: vertices, then dual edges (1D),
 * faces (2D) and interiors (3D) by exact local solves, one workgroup per
 * dual region.  Pressure independent: built once per rock.
 * Errors: CAMS_E_STATE (no rock), CAMS_E_BREAKDOWN (non-positive pivot). */
cams_status cams_build_basis(cams_ctx *ctx);

/* Coarse operator A_c = R A P_hat (Eq. (13); P_hat = basis with Dirichlet rows
 * zeroed, R = R^FV of Eq. (7) or P_hat^T) and the explicit inverse used by
 * every coarse solve: MSFV by LU with partial pivoting; MSFE (symmetric
 * positive definite) by Gauss-Jordan sweeps without pivoting, or, above 4096
 * coarse nodes with at least 3 coarse z-planes, by block elimination over
 * the z-planes (one dense inverse per plane) from both ends towards the
 * middle plane, the two chains at the same time on two streams.
 * Errors: CAMS_E_STATE (no basis or no assembled system), CAMS_E_BREAKDOWN
 * (singular coarse matrix). */
cams_status cams_coarse_op(cams_ctx *ctx);

/* Solve the assembled system for the Newton update by C-AMS iterations
 * (Table "cams"; Eq. (15) multiscale stage, ILU(0) smoothing) and add it to
 * p_dev in place:  p <- p + d,  A d = r.  Stops when
 * ||r||_2 <= max(lin_rtol ||r0||_2, lin_atol) or after lin_maxit iterations.  Stagnation
 * also stops it: when ||r||_2 has not fallen below 0.9 times its smallest
 * value so far for 100 iterations (e.g. a tolerance below the rounding level
 * of the FP64 residual).  `stats` may be NULL.  Errors: CAMS_E_STATE (no
 * coarse operator for the current system), CAMS_E_NOT_CONVERGED (limit
 * reached or stagnation; p holds the last iterate whose residual was
 * evaluated), CAMS_E_BREAKDOWN (non-finite residual norm). */
cams_status cams_iterate(cams_ctx *ctx, double *p_dev, cams_stats *stats);

/* One backward-Euler time step: Dirichlet values are imposed on p_dev, the
 * basis is built if needed, then repeat assemble -> (stop if ||eps||_2 <=
 * newton_tol) -> coarse_op -> iterate, at most newton_maxit solves.
 * p_dev (in/out) starts as the initial guess (normally pn_dev).
 * Errors: as the calls above; CAMS_E_NOT_CONVERGED if Newton does not reach
 * newton_tol. */
cams_status cams_newton_step(cams_ctx *ctx, const double *pn_dev, double *p_dev, cams_stats *stats);

/* Mass-conservative finish of a time step (Sec. 4.2: converge with MSFE,
 * then apply a single MSFV sweep; an MSFV stage yields fluxes that are
 * conservative on the coarse grid, Sec. 4).  At pressure p_dev (normally
 * the converged result of cams_newton_step with MSFE) and old-time pressure
 * pn_dev: assemble the Newton system (Eqs. (3)-(6)), form the MSFV coarse
 * operator R^FV A P_hat (Eqs. (7), (13)), invert it (LU with partial
 * pivoting), and apply one multiscale stage d = P_hat (R^FV A P_hat)^-1 R^FV r
 * (Eqs. (12), (15)); p_dev += d.  flux_dev (3N doubles, device) receives
 * the two-point mass fluxes of that linear system at the updated pressure,
 * T (rho(p_n) + rho(p_m))/2 (p'_n - p'_m) with the face densities of the
 * assembly point p and the updated p', on the +x, +y, +z face of every cell
 * (positive out of the cell, 0 on the domain boundary): on every primal
 * coarse block, accumulation (linearised at p) + net outflow - sources sums
 * to zero.  Builds the basis if needed; the coarse factorisation is
 * replaced, so the next cams_iterate needs cams_coarse_op again.
 * Errors: CAMS_E_STATE (no rock), CAMS_E_ARG (null arrays; more than 4096
 * coarse nodes, which use the block-tridiagonal MSFE factorisation),
 * CAMS_E_BREAKDOWN (singular coarse matrix), CAMS_E_DEVICE. */
cams_status cams_conservative_sweep(cams_ctx *ctx, const double *pn_dev, double *p_dev, double *flux_dev);

/* One time step as cams_newton_step, recording after every C-AMS iteration
 * (each evaluation of the linear residual, the first one being r0) the
 * Newton iteration index nu, the linear residual norm ||r||_2 of the
 * current Newton system and the nonlinear error ||eps||_2 (Eq. (16)) at the
 * current iterate p^nu + d.  These are the error and residual norm histories
 * of the paper's study of linear and nonlinear stopping (Sec. 4.1.1: with
 * the linear solve converged at every Newton step, and with the adaptive
 * strategy of lin_rtol = 1e-1 and newton_tol = 1e-6, which updates the
 * linear system only after the residual has dropped by an order of
 * magnitude).  Host arrays of `cap` entries receive the first `cap` entries;
 * *count is set to the number of entries produced (may exceed cap).  Each
 * entry costs one extra nonlinear-error evaluation and a synchronisation:
 * for studies, not for timing.  Errors: as cams_newton_step; CAMS_E_ARG
 * (null buffers with cap > 0, null count). */
cams_status cams_newton_history(cams_ctx *ctx, const double *pn_dev, double *p_dev, double *res_host,
                                double *err_host, int32_t *newton_host, int32_t cap, int32_t *count,
                                cams_stats *stats);

/* One application of the smoother, x = M^{-1} z, with M the ILU(0) factor of
 * the assembled matrix chosen by options.smoother (Table "cams" step 6); for
 * BLOCK_ALT the pair of Richardson steps from zero, x1 = M0^{-1} z and
 * x = x1 + M1^{-1}(z - A x1) (M0: blocks at the origin, M1: shifted).  z_dev and
 * x_dev have N entries.  Errors: CAMS_E_STATE (no coarse_op for the current
 * system: the factor is computed there). */
cams_status cams_smooth_apply(cams_ctx *ctx, const double *z_dev, double *x_dev);

/* Copy an internal array to dst_dev (device, `bytes` >= cams_array_bytes).
 * For inspection and parity tests.  Errors: CAMS_E_ARG, CAMS_E_STATE. */
typedef enum {
    CAMS_ARR_T = 0,        /* 3*N doubles: Tx, Ty, Tz (face on its lower cell) */
    CAMS_ARR_W = 1,        /* 3*N doubles: masked off-diagonal magnitudes of A */
    CAMS_ARR_DIAG = 2,     /* N doubles */
    CAMS_ARR_R0 = 3,       /* N doubles: Newton residual r = -F */
    CAMS_ARR_P = 4,        /* 8*N doubles: basis weights, slot-major */
    CAMS_ARR_AC = 5,       /* Nc*Nc doubles: coarse operator, row-major (before factorisation) */
    CAMS_ARR_AC_INV = 6,   /* Nc*Nc doubles: inverse of the coarse operator */
    CAMS_ARR_INVD = 7      /* N doubles: inverse ILU(0) pivots of the smoother (2N for BLOCK_ALT:
                              those of the shifted block grid follow) */
} cams_array;

size_t cams_array_bytes(const cams_ctx *ctx, cams_array which);
cams_status cams_export(cams_ctx *ctx, cams_array which, void *dst_dev, size_t bytes);
/* Replace the basis by a saved one: src_dev holds 8*N doubles on the device,
 * slot-major as CAMS_ARR_P exports them, bytes = cams_array_bytes(ctx,
 * CAMS_ARR_P).  For resuming a run from a checkpoint without rebuilding the
 * basis: types B3 and B4 only, whose basis depends on the rock and not on
 * the pressure (Sec. 3).  The mixed precisions round it as after a build;
 * the next cams_coarse_op uses it.  The caller vouches that it belongs to
 * the current rock.  Errors: CAMS_E_ARG (null, size, basis type B1/B2),
 * CAMS_E_STATE (no rock), CAMS_E_DEVICE. */
cams_status cams_import_basis(cams_ctx *ctx, const void *src_dev, size_t bytes);

/* Test hook of the coarse factorisation's FP64 matrix-core GEMM: C -= A B for
 * dense row-major DEVICE matrices C (M x Nn), A (M x K), B (K x Nn), run on the
 * context's stream and synchronised.  Used by the parity tests of the blocked
 * LU (Sec. 3, coarse solve of Eq. (15)).  Errors: CAMS_E_ARG, CAMS_E_DEVICE. */
cams_status cams_debug_gemm_sub(cams_ctx *ctx, double *C_dev, const double *A_dev, const double *B_dev,
                                int M, int Nn, int K);

/* Measurement hook: time every launch of one kernel class with HIP events on
 * the context's stream (kernel = CAMS_PROF_SMOOTH_STEP, the block-ILU(0)
 * Richardson step of Table "cams" step 6; CAMS_PROF_NONE switches timing off
 * and clears the totals).  To keep the event overhead out of the run, only
 * the smoothing sequences of every 16th C-AMS iteration are timed, each as
 * one bracket around its back-to-back launches (so the time includes the
 * short gaps between them); iterations past convergence are not counted.  cams_profile_read returns the
 * summed device time in ms, the number of counted launches and their summed
 * algorithmic bytes (each array read or written once per launch).
 * Errors: CAMS_E_ARG, CAMS_E_DEVICE. */
enum { CAMS_PROF_NONE = 0, CAMS_PROF_SMOOTH_STEP = 1 };
cams_status cams_profile(cams_ctx *ctx, int kernel);
cams_status cams_profile_read(cams_ctx *ctx, double *total_ms, int64_t *launches, double *bytes);

/* ---- Learned basis (extension of the basis construction of Sec. 3) ------
 * A 3D CNN maps the log-transmissibility patch of a full dual block (the
 * 9x9x9 cells between and on its bounding vertex planes; ratio 8, 3D only)
 * to the 8 basis values of its 7x7x7 interior cells; a softmax over the 8
 * vertex channels makes the prediction a partition of unity.  Features:
 * channel 0/1/2 = ln T on each patch cell's +x/+y/+z face (0 on the patch's
 * last face of that axis), layout feat[b][c][x + 9(y + 9z)] float.  Network:
 * conv3d 3->32, ReLU, 32->32, ReLU, 32->32, ReLU, 32->8, 3x3x3 kernels, zero
 * padding; parameters one float vector, per layer W[tap][ci][co] (tap =
 * 9(dz+1) + 3(dy+1) + (dx+1)) followed by the bias[co].  Outputs phi[b][s][p]
 * (s = corner bx + 2by + 4bz of the block), targets tgt[b][s][x + 7(y + 7z)]
 * over the interior cells.  All arrays are device memory, FP32. */

/* Number of network parameters (64904). */
int64_t cams_cnn_num_params(void);
/* Scratch bytes the network calls below need for a batch of `batch` patches. */
size_t cams_cnn_workspace_bytes(int32_t batch);
/* phi = network(feat) for `batch` patches, on `stream` (hipStream_t).
 * Errors: CAMS_E_ARG (null pointer, batch <= 0), CAMS_E_DEVICE. */
cams_status cams_cnn_forward(void *stream, const float *params_dev, const float *feat_dev, int32_t batch,
                             void *ws_dev, float *phi_dev);
/* The same network on matrix cores: the parameters are converted to
 * bfloat16 (weights; biases stay FP32) into ws_dev (at least
 * cams_cnn_bf16_workspace_bytes(), 16-byte aligned), activations are
 * bfloat16 between layers, every product accumulates in FP32 (one workgroup
 * per patch, v_mfma_f32_16x16x32_bf16).  This is what cams_build_basis uses
 * for the learned interiors.  Errors: CAMS_E_ARG, CAMS_E_DEVICE. */
size_t cams_cnn_bf16_workspace_bytes(void);
cams_status cams_cnn_forward_bf16(void *stream, const float *params_dev, const float *feat_dev, int32_t batch,
                                  void *ws_dev, float *phi_dev);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid allocation): cams_cnn_forward_bf16
 * without the caller's workspace.  The bfloat16 weights and FP32 biases are
 * staged in a fixed device array of cams_cnn_noalloc_scratch_bytes() bytes
 * (512 KB) that each GPU the library runs on holds until the process ends;
 * its address on the current device is looked up once (the stream must
 * belong to the current device).  Calls allocate nothing.  Every call on a
 * GPU shares that GPU's array and rewrites it from `params_dev`, so calls
 * that overlap on one GPU (different streams, or threads) race.  Same
 * arguments and result as cams_cnn_forward_bf16.
 * Errors: CAMS_E_ARG (null pointer, batch <= 0), CAMS_E_NOMEM (the network
 * needs more than the fixed array), CAMS_E_DEVICE. */
size_t cams_cnn_noalloc_scratch_bytes(void);
cams_status cams_cnn_forward_bf16_noalloc(void *stream, const float *params_dev, const float *feat_dev,
                                          int32_t batch, float *phi_dev);
/* Mean-squared error of phi against tgt over the interior cells and 8 channels
 * (written to *loss_dev, a device double) and its gradient wrt the
 * parameters (grad_dev, cams_cnn_num_params floats); the project's own
 * backward kernels.  Errors: CAMS_E_ARG, CAMS_E_DEVICE. */
cams_status cams_cnn_loss_grad(void *stream, const float *params_dev, const float *feat_dev, const float *tgt_dev,
                               int32_t batch, void *ws_dev, float *grad_dev, double *loss_dev);
/* One bias-corrected Adam update of n parameters at step `step` (>= 1).
 * Errors: CAMS_E_ARG, CAMS_E_DEVICE. */
cams_status cams_cnn_adam(void *stream, float *params_dev, const float *grad_dev, float *m_dev, float *v_dev,
                          int32_t n, int32_t step, float lr, float beta1, float beta2, float eps);
/* Number of full dual blocks of the context (those the network handles). */
int32_t cams_cnn_num_blocks(const cams_ctx *ctx);
/* Training patches of the context: features of every full dual block, and
 * (tgt_dev non-NULL, basis built) the exact basis values of its interior.
 * Synchronises.  Errors: CAMS_E_ARG, CAMS_E_STATE (no rock / no basis). */
cams_status cams_cnn_patches(cams_ctx *ctx, float *feat_dev, float *tgt_dev);
/* Scratch bytes cams_set_learned needs for this context. */
size_t cams_learned_scratch_bytes(const cams_ctx *ctx);
/* Switch cams_build_basis to the learned interiors (params_dev non-NULL) or
 * back to exact local solves (NULL).  Edges, faces and stub interiors stay
 * exact; each predicted interior is checked with the local equation, and a
 * block with ||(T Phi)_I|| / ||T_IF Phi_F|| > fallback_tol is re-solved
 * exactly.  params_dev and scratch_dev (256-byte aligned) are borrowed until
 * switched off.  Invalidates the basis.  Errors: CAMS_E_ARG (not 3D with
 * ratio 8, scratch too small, fallback_tol <= 0). */
cams_status cams_set_learned(cams_ctx *ctx, const float *params_dev, void *scratch_dev, size_t scratch_bytes,
                             double fallback_tol);
/* Global check of the learned basis, beside the per-block one: plain_iters
 * is the number of C-AMS iterations per Newton linear solve that the exact
 * (local-solve) basis needs on this problem, measured by the caller (0, the
 * default, switches the check off).  When a linear solve of
 * cams_newton_step with the learned basis takes more than 2 * plain_iters
 * iterations, or stops without converging, the basis is rebuilt with local
 * solves; the Newton iteration goes on from the iterate reached, and the
 * rest of the time step and every later one use the exact basis
 * (stats.basis_rebuilds counts the rebuild).  The learned basis comes back
 * with the next cams_set_learned or cams_set_rock.
 * Errors: CAMS_E_ARG (plain_iters < 0). */
cams_status cams_set_learned_guard(cams_ctx *ctx, int32_t plain_iters);
/* Blocks taken from the network and blocks re-solved by the fallback in the
 * last cams_build_basis.  Errors: CAMS_E_ARG. */
/* The local-equation ratio ||(T Phi)_I|| / ||T_IF Phi_F|| of the network's
 * prediction for each full dual block of the last learned cams_build_basis
 * (before any fallback), in block order (x fastest); n <= the number of full
 * blocks, written to host memory.  Used to calibrate fallback_tol.
 * Errors: CAMS_E_ARG, CAMS_E_STATE (no learned build, or n too large). */
cams_status cams_basis_block_ratios(const cams_ctx *ctx, double *ratio_host, int32_t n);
cams_status cams_basis_stats(const cams_ctx *ctx, int32_t *learned_blocks, int32_t *fallback_blocks);

/* Number of coarse nodes (product of ceil(n/r) per axis). */
int64_t cams_num_coarse(const cams_ctx *ctx);

/* Coarse factorisation layout.  The MSFE coarse operator couples only nodes
 * of adjacent z-planes of the coarse grid (a basis function of Eq. (11)
 * vanishes on the vertex planes beside its own), so for 3D grids with more
 * than 4096 coarse nodes and at least 3 planes it is factorised by block
 * elimination over the planes (Schur complements S_k = D_k - L_k S_{k-1}^-1
 * U_{k-1}, each inverted densely) instead of one dense inversion.  Returns
 * the number of planes in that case, 0 for the dense explicit inverse. */
int32_t cams_coarse_planes(const cams_ctx *ctx);

/* Test hook: xc_dev = A_c^-1 rc_dev (Nc device doubles each) with the
 * factorisation of the last cams_coarse_op.  Synchronises. */
cams_status cams_debug_coarse_solve(cams_ctx *ctx, const double *rc_dev, double *xc_dev);

cams_status cams_destroy(cams_ctx *ctx);
const char *cams_status_string(cams_status s);
const char *cams_last_error(const cams_ctx *ctx);

/* ---- Batched solve of many independent problems.
 *
 * One Newton iteration of Sec. 2 (assembly of Eqs. (3)-(6), basis of
 * Eq. (11) if not built yet, coarse system of Eq. (13), C-AMS iterations of
 * Table "cams" to lin_rtol, update p += delta) for every context of the
 * batch at once.  Each C-AMS iteration is one launch per kernel over the
 * cells of ALL instances; instances that have met their stopping test stop
 * taking part.  The iterations run from HIP graphs captured at the first
 * call; the smoother's workgroup size and the number of iterations per
 * graph are tuned on that call by timing (cams_batch_tuning reports them).
 *
 * The contexts must have been created on the same stream (the one given
 * here), have their workspace and rock set, share precision and n_pre /
 * n_post, use a block ILU(0) smoother (BLOCK or BLOCK_ALT, may differ per
 * instance) and the local basis (no learned
 * basis).  The batch keeps pointers to the contexts: destroy it before them.
 * Each instance computes exactly what cams_newton_step with newton_maxit = 1
 * computes for its first linear solve (same kernels, same order of
 * floating-point operations within an instance).
 */
typedef struct cams_batch cams_batch;

/* Group `count` contexts; builds the host work lists.  No HIP call.
 * Errors: CAMS_E_ARG (null/duplicate context, different stream, precision
 * or smoothing counts, red-black smoother), CAMS_E_NOMEM. */
cams_status cams_batch_create(cams_ctx *const *ctxs, int32_t count, void *hip_stream, cams_batch **out);
/* Device workspace of the batch (instance table, work lists, counters). */
size_t cams_batch_workspace_bytes(const cams_batch *b);
/* Attach the batch workspace (device memory, 256-byte aligned, caller
 * owned, must outlive the batch) and upload the tables; call again after a
 * context's workspace changes.  Creates the batch's own streams, events and
 * a small pinned host buffer at the first call.  Synchronises. */
cams_status cams_batch_set_workspace(cams_batch *b, void *ws_dev, size_t bytes);
/* One Newton iteration for every instance.  pn_dev[i], p_dev[i]: device
 * pressures of instance i (p_dev[i] is updated in place).  status_out[i]
 * (nullable): CAMS_OK, CAMS_E_NOT_CONVERGED (lin_maxit reached) or
 * CAMS_E_BREAKDOWN.  stats[i] (nullable): newton_iters = 1, C-AMS
 * iterations, relative residual, ||eps|| of the assembled iterate,
 * t_coarse_ms = wall time of the overlapped setup phases of the batch,
 * t_iterate_ms = wall time of the batched iterations.  Returns CAMS_OK when
 * every instance succeeded, else the first failing instance's status.
 * Synchronises. */
cams_status cams_batch_newton_iteration(cams_batch *b, const double *const *pn_dev, double *const *p_dev,
                                        int32_t *status_out, cams_stats *stats);
/* Tuning outcome (0 / unset before the first call): iterations per graph
 * replay, and the smoother's workgroup: threads per workgroup and 8x8x8
 * blocks per workgroup (1, or 4 neighbouring blocks along x); with the
 * measured ms per batched iteration of the graph candidates (2, 4, 8
 * iterations per graph, up to 3 entries) and ms per smoothing step of the
 * smoother candidates (128, 256, 512 threads per block, then 4 blocks per
 * 512 threads, FP32 only and 0 when not measured; up to 4 entries); at most
 * `ncand` entries of each array are written (pointers nullable). */
cams_status cams_batch_tuning(const cams_batch *b, int32_t *iters_per_graph, int32_t *smoother_threads,
                              int32_t *smoother_blocks, double *ms_per_iter_candidates,
                              double *ms_per_smooth_step_candidates, int32_t ncand);
/* Fix the smoother form instead of the tuner's choice: `threads` per
 * workgroup and `blocks` 8x8x8 blocks per workgroup, one of (128, 1),
 * (256, 1), (512, 1) and, in mixed precision, (512, 4); (0, 0) returns to
 * the tuned choice.  The iterations are captured (and the graph length
 * tuned) again on the next call.  For reproducible timings and for tests
 * of each form.  Errors: CAMS_E_ARG (another pair). */
cams_status cams_batch_set_smoother(cams_batch *b, int32_t threads, int32_t blocks);
/* The tuning outcome is kept per process, keyed by precision, n_pre,
 * n_post, whether an instance alternates block grids, and floor(log2) of
 * the batch's total cells and of its instance count: a later batch with the
 * same key takes the stored choice (and its timings, for cams_batch_tuning)
 * instead of timing the candidates.  *from_cache: 1 when the batch's
 * current choice came from there, 0 when it was measured (and stored), -1
 * before the first call or with a smoother fixed by cams_batch_set_smoother.
 * Errors: CAMS_E_ARG (null). */
cams_status cams_batch_tuning_source(const cams_batch *b, int32_t *from_cache);
/* Forget every stored tuning outcome (later batches measure again). */
void cams_batch_clear_tuning_cache(void);
const char *cams_batch_last_error(const cams_batch *b);
void cams_batch_destroy(cams_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* CAMS_H */
