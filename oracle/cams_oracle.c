/*
 * CPU oracle for the C-AMS pressure solve — TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 implementation of what the compressible algebraic
 * multiscale solver (Tene, Wang, Hajibeygi, arXiv 1705.05783) computes.  Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * call it; the GPU library shares no code with it.
 *
 * Equations are numbered in order of appearance in the paper:
 *   (1) mass balance, (2) semi-discrete nonlinear pressure equation,
 *   (3) linearisation, (4) accumulation coefficient c^nu, (5) rhs b^nu,
 *   (6) algebraic system A p = f, (7) finite-volume restriction,
 *   (8)-(11) basis equations B1..B4, (12) superposition p' = P p_coarse,
 *   (13) coarse system R A P, (14)-(15) multiscale solution / correction,
 *   (16) nonlinear error epsilon.  Table "cams" is the iteration procedure.
 *
 * Readings taken where the paper is silent (each also listed in the design
 * notes of the repository):
 *   - rho(p) = rho0 exp(c (p - p0)); porosity constant in time;
 *   - two-point flux with harmonic averaging of cell conductances, face
 *     density = arithmetic mean of the two cell densities;
 *   - equations (2)/(3) are multiplied by rho_i dV_i ("mass form"), which
 *     leaves the Newton update unchanged and makes the matrix symmetric;
 *   - wells are Dirichlet cells: identity rows/columns, zero residual;
 *   - reduced-problem boundary conditions of the basis (Sec. 3) follow the
 *     wirebasket algebra of the AMS paper the authors cite: couplings to
 *     lower-dimensional neighbours are lumped onto the diagonal;
 *   - vertex of a primal block of length L starting at s is s + floor(L/2).
 *
 * Parity status per function is listed in the header comment of each.
 *
 * The tests build this file without OpenMP, so every "omp" pragma below is
 * ignored there and the oracle runs serially and deterministically.  The
 * CPU-baseline timing build (-O3 -march=native -fopenmp) runs the loops the
 * pragmas mark on all host cores: cells, dual regions of one level, rows of
 * the coarse LU update, blocks of a block-ILU(0) factor.  Only reductions
 * and the scatter-adds of the coarse operator and the restriction change
 * their order of summation there.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;
    int32_t rx, ry, rz;
} og_grid;

typedef struct {
    double rho0, c, p0, mu, dt;
} og_fluid;

#define OR_FV 0
#define OR_FE 1

static long cell_index(const og_grid *g, int i, int j, int k)
{
    return (long)i + (long)g->nx * ((long)j + (long)g->ny * (long)k);
}

static long ncells(const og_grid *g) { return (long)g->nx * g->ny * g->nz; }

/* The six neighbours of a cell through its faces.  For face f of cell n the
 * neighbour index and the face transmissibility are returned; faces on the
 * domain boundary have no neighbour (no-flow, Sec. 4). */
static int neighbour(const og_grid *g, const double *Tx, const double *Ty, const double *Tz,
                     long n, int f, long *m, double *T)
{
    int i = (int)(n % g->nx);
    int j = (int)((n / g->nx) % g->ny);
    int k = (int)(n / ((long)g->nx * g->ny));
    switch (f) {
    case 0: if (i == 0) return 0; *m = n - 1; *T = Tx[n - 1]; return 1;
    case 1: if (i == g->nx - 1) return 0; *m = n + 1; *T = Tx[n]; return 1;
    case 2: if (j == 0) return 0; *m = n - g->nx; *T = Ty[n - g->nx]; return 1;
    case 3: if (j == g->ny - 1) return 0; *m = n + g->nx; *T = Ty[n]; return 1;
    case 4: if (k == 0) return 0; *m = n - (long)g->nx * g->ny; *T = Tz[n - (long)g->nx * g->ny]; return 1;
    case 5: if (k == g->nz - 1) return 0; *m = n + (long)g->nx * g->ny; *T = Tz[n]; return 1;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Two-point flux transmissibility (Sec. 2, Eq. (6): the matrix entries are
 * fine-scale transmissibilities of a finite-volume scheme).  Each face
 * conductance is the series combination of the two half-cell conductances
 * lambda A / (h/2), lambda = k / mu.  Stored on the lower cell of the face;
 * faces on the domain boundary are zero.
 * Pinned: homogeneous closed form, 1D series resistance.
 * ---------------------------------------------------------------------- */
void or_transmissibility(const og_grid *g, double mu, const double *perm,
                         double *Tx, double *Ty, double *Tz)
{
    double ax = g->dy * g->dz, ay = g->dx * g->dz, az = g->dx * g->dy;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < g->nz; k++)
        for (int j = 0; j < g->ny; j++)
            for (int i = 0; i < g->nx; i++) {
                long n = cell_index(g, i, j, k);
                double lam = perm[n] / mu;
                Tx[n] = Ty[n] = Tz[n] = 0.0;
                if (i + 1 < g->nx) {
                    double a = lam * ax / (g->dx / 2), b = (perm[n + 1] / mu) * ax / (g->dx / 2);
                    Tx[n] = 1.0 / (1.0 / a + 1.0 / b);
                }
                if (j + 1 < g->ny) {
                    long m = n + g->nx;
                    double a = lam * ay / (g->dy / 2), b = (perm[m] / mu) * ay / (g->dy / 2);
                    Ty[n] = 1.0 / (1.0 / a + 1.0 / b);
                }
                if (k + 1 < g->nz) {
                    long m = n + (long)g->nx * g->ny;
                    double a = lam * az / (g->dz / 2), b = (perm[m] / mu) * az / (g->dz / 2);
                    Tz[n] = 1.0 / (1.0 / a + 1.0 / b);
                }
            }
}

static double density(const og_fluid *f, double p) { return f->rho0 * exp(f->c * (p - f->p0)); }

/* ------------------------------------------------------------------------
 * Nonlinear residual of the backward-Euler pressure equation (Sec. 2,
 * Eq. (2)), multiplied by rho_i dV_i:
 *   F_i = phi_i dV (rho_i - rho_i^n)/dt + sum_j T_ij rho_ij (p_i - p_j) - rho_i q_i dV
 * with rho_ij the mean of the two cell densities.  F_i = 0 on Dirichlet cells.
 * A Dirichlet boundary face (fixed pressure pb on the west or east face,
 * Sec. 4: the default test cases) adds T_b (rho_i + rho(pb))/2 (p_i - pb),
 * with T_b = 2 lambda_i A / dx the half-cell transmissibility between the
 * cell centre and the face: bt[i] = T_b, bp[i] = pb (both NULL: no face
 * condition; bt[i] = 0 on cells without one).
 * The nonlinear error (Sec. 4.1.1, Eq. (16)) is eps_i = F_i / (rho_i dV);
 * the function returns ||eps||_2 over the non-Dirichlet cells.
 * Pinned: global mass balance, c = 0 linearity, direct-solve Newton.
 * ---------------------------------------------------------------------- */
double or_nonlinear_residual(const og_grid *g, const og_fluid *f,
                             const double *Tx, const double *Ty, const double *Tz,
                             const double *phi, const double *q, const uint8_t *dmask,
                             const double *bt, const double *bp,
                             const double *p, const double *pn, double *F)
{
    long N = ncells(g);
    double dV = g->dx * g->dy * g->dz, e2 = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : e2)
    for (long n = 0; n < N; n++) {
        if (dmask[n]) { F[n] = 0.0; continue; }
        double rho = density(f, p[n]), rhon = density(f, pn[n]);
        double acc = phi[n] * dV * (rho - rhon) / f->dt;
        double flux = 0.0;
        for (int fc = 0; fc < 6; fc++) {
            long m; double T;
            if (!neighbour(g, Tx, Ty, Tz, n, fc, &m, &T)) continue;
            double rhof = 0.5 * (rho + density(f, p[m]));
            flux += T * rhof * (p[n] - p[m]);
        }
        if (bt && bt[n] > 0.0) flux += bt[n] * 0.5 * (rho + density(f, bp[n])) * (p[n] - bp[n]);
        double src = q ? rho * q[n] * dV : 0.0;
        F[n] = acc + flux - src;
        double e = F[n] / (rho * dV);
        e2 += e * e;
    }
    return sqrt(e2);
}

/* ------------------------------------------------------------------------
 * Linear system of one Newton-Raphson iteration (Sec. 2, Eqs. (3)-(6)),
 * scaled by rho_i^nu dV_i and written for the update d = p^{nu+1} - p^nu:
 *   A d = r,  A_ii = c_i^nu rho_i^nu dV + sum_j W_ij,  A_ij = -W_ij,  r = -F(p^nu)
 * where W_ij = T_ij (rho_i^nu + rho_j^nu)/2 and, with constant porosity,
 * c_i^nu rho_i^nu dV = phi_i c rho_i^n dV / dt (Eq. (4)).  Dirichlet rows and
 * columns are identity: W is zeroed on faces touching a Dirichlet cell (the
 * diagonal of the free neighbour keeps the coupling), A_DD = 1, r_D = 0.
 * Output: masked off-diagonal magnitudes Wx/Wy/Wz on the lower cell of each
 * face, the diagonal, and r.  Returns ||eps||_2.
 * Pinned: symmetry/M-matrix, finite-difference Jacobian of the
 * frozen-density residual at p = p^n, c = 0 exactness.
 * ---------------------------------------------------------------------- */
double or_linear_system(const og_grid *g, const og_fluid *f,
                        const double *Tx, const double *Ty, const double *Tz,
                        const double *phi, const double *q, const uint8_t *dmask,
                        const double *bt, const double *bp,
                        const double *p, const double *pn,
                        double *Wx, double *Wy, double *Wz, double *diag, double *r)
{
    long N = ncells(g);
    double dV = g->dx * g->dy * g->dz;
    double en = or_nonlinear_residual(g, f, Tx, Ty, Tz, phi, q, dmask, bt, bp, p, pn, r);
    for (long n = 0; n < N; n++) r[n] = -r[n];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < g->nz; k++)
        for (int j = 0; j < g->ny; j++)
            for (int i = 0; i < g->nx; i++) {
                long n = cell_index(g, i, j, k);
                double rho = density(f, p[n]);
                Wx[n] = Wy[n] = Wz[n] = 0.0;
                if (i + 1 < g->nx && !dmask[n] && !dmask[n + 1])
                    Wx[n] = Tx[n] * 0.5 * (rho + density(f, p[n + 1]));
                if (j + 1 < g->ny && !dmask[n] && !dmask[n + g->nx])
                    Wy[n] = Ty[n] * 0.5 * (rho + density(f, p[n + g->nx]));
                long s = (long)g->nx * g->ny;
                if (k + 1 < g->nz && !dmask[n] && !dmask[n + s])
                    Wz[n] = Tz[n] * 0.5 * (rho + density(f, p[n + s]));
                if (dmask[n]) { diag[n] = 1.0; continue; }
                double d = phi[n] * f->c * density(f, pn[n]) * dV / f->dt;
                for (int fc = 0; fc < 6; fc++) {
                    long m; double T;
                    if (!neighbour(g, Tx, Ty, Tz, n, fc, &m, &T)) continue;
                    d += T * 0.5 * (rho + density(f, p[m]));
                }
                if (bt && bt[n] > 0.0) d += bt[n] * 0.5 * (rho + density(f, bp[n]));
                diag[n] = d;
            }
    return en;
}

/* ------------------------------------------------------------------------
 * Two-point mass fluxes (Sec. 2, the flux term of Eqs. (2)-(3)): on the face
 * between cell n and its +x / +y / +z neighbour m,
 *   flux = T_nm (rho(q_n) + rho(q_m)) / 2 (p_n - p_m),
 * positive from n to m, stored on n (0 on the domain boundary).  With q = p
 * these are the fluxes of the nonlinear residual F; with q the iterate at
 * which a Newton system was assembled and p its updated solution they are
 * the fluxes of that linear system (face densities frozen at q).
 * Pinned: F rebuilt from the fluxes equals or_nonlinear_residual; after an
 * MSFV stage the coarse-block sums of the linearised balance vanish.
 * ---------------------------------------------------------------------- */
void or_face_flux(const og_grid *g, const og_fluid *f, const double *Tx, const double *Ty, const double *Tz,
                  const double *q, const double *p, double *Fx, double *Fy, double *Fz)
{
    long s = (long)g->nx * g->ny;
    for (int k = 0; k < g->nz; k++)
        for (int j = 0; j < g->ny; j++)
            for (int i = 0; i < g->nx; i++) {
                long n = cell_index(g, i, j, k);
                double rho = density(f, q[n]);
                Fx[n] = Fy[n] = Fz[n] = 0.0;
                if (i + 1 < g->nx) Fx[n] = Tx[n] * 0.5 * (rho + density(f, q[n + 1])) * (p[n] - p[n + 1]);
                if (j + 1 < g->ny) Fy[n] = Ty[n] * 0.5 * (rho + density(f, q[n + g->nx])) * (p[n] - p[n + g->nx]);
                if (k + 1 < g->nz) Fz[n] = Tz[n] * 0.5 * (rho + density(f, q[n + s])) * (p[n] - p[n + s]);
            }
}

/* y = A x for the 7-point operator stored as (W, diag). */
void or_matvec(const og_grid *g, const double *Wx, const double *Wy, const double *Wz,
               const double *diag, const double *x, double *y)
{
    long N = ncells(g);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; n++) {
        double s = diag[n] * x[n];
        for (int fc = 0; fc < 6; fc++) {
            long m; double W;
            if (!neighbour(g, Wx, Wy, Wz, n, fc, &m, &W)) continue;
            s -= W * x[m];
        }
        y[n] = s;
    }
}

/* ------------------------------------------------------------------------
 * Primal / dual coarse grids (Sec. 3, figure "msfv-grid").
 * Along each axis the primal blocks are [a r, min((a+1) r, n) - 1] and the
 * coarse node (vertex) of block a sits at a r + floor(len_a / 2).  The dual
 * grid is formed by the lines/planes through the vertices.  A cell's level is
 * the number of active axes on which its coordinate is a vertex coordinate
 * (3D: 3 vertex, 2 edge, 1 face, 0 interior; 2D: 2 vertex, 1 edge, 0
 * interior).
 * ---------------------------------------------------------------------- */
int or_num_blocks(int n, int r) { return (n + r - 1) / r; }

void or_vertex_coords(int n, int r, int32_t *v)
{
    int nb = or_num_blocks(n, r);
    for (int a = 0; a < nb; a++) {
        int s = a * r, e = (a + 1) * r < n ? (a + 1) * r : n;
        v[a] = s + (e - s) / 2;
    }
}

typedef struct {
    int nb[3];
    int32_t *vc[3];     /* vertex coordinates per axis */
    int32_t *isv[3];    /* is-vertex flag per coordinate */
    int32_t *lo[3];     /* lower bracketing vertex per coordinate */
    int dim;
} og_dual;

static void dual_init(const og_grid *g, og_dual *d)
{
    int n[3] = {g->nx, g->ny, g->nz}, r[3] = {g->rx, g->ry, g->rz};
    d->dim = g->nz > 1 ? 3 : 2;
    for (int a = 0; a < 3; a++) {
        d->nb[a] = or_num_blocks(n[a], r[a]);
        d->vc[a] = (int32_t *)malloc(sizeof(int32_t) * d->nb[a]);
        d->isv[a] = (int32_t *)calloc(n[a], sizeof(int32_t));
        d->lo[a] = (int32_t *)malloc(sizeof(int32_t) * n[a]);
        or_vertex_coords(n[a], r[a], d->vc[a]);
        for (int b = 0; b < d->nb[a]; b++) d->isv[a][d->vc[a][b]] = 1;
        for (int x = 0; x < n[a]; x++) {
            int lo = 0;
            for (int b = 0; b < d->nb[a]; b++)
                if (d->vc[a][b] <= x) lo = b;
            d->lo[a][x] = lo;
        }
    }
}

static void dual_free(og_dual *d)
{
    for (int a = 0; a < 3; a++) { free(d->vc[a]); free(d->isv[a]); free(d->lo[a]); }
}

static int cell_level(const og_grid *g, const og_dual *d, long n)
{
    int i = (int)(n % g->nx), j = (int)((n / g->nx) % g->ny), k = (int)(n / ((long)g->nx * g->ny));
    int L = d->isv[0][i] + d->isv[1][j];
    if (d->dim == 3) L += d->isv[2][k];
    return L;
}

/* Levels of all cells (for the pins). */
void or_cell_levels(const og_grid *g, int32_t *level)
{
    og_dual d; dual_init(g, &d);
    for (long n = 0; n < ncells(g); n++) level[n] = cell_level(g, &d, n);
    dual_free(&d);
}

/* Coarse node index and slot of coarse node (a,b,c) as seen from cell n; the
 * slot is the position of the node among the (up to) 2x2x2 vertices that
 * bracket the cell.  Returns -1 if the node is not a bracketing vertex. */
static int node_slot(const og_grid *g, const og_dual *d, long n, int a, int b, int c)
{
    int i = (int)(n % g->nx), j = (int)((n / g->nx) % g->ny), k = (int)(n / ((long)g->nx * g->ny));
    int sx = a - d->lo[0][i], sy = b - d->lo[1][j], sz = c - d->lo[2][k];
    if (sx < 0 || sx > 1 || sy < 0 || sy > 1 || sz < 0 || sz > 1) return -1;
    return sx + 2 * sy + 4 * sz;
}

static long node_of_slot(const og_grid *g, const og_dual *d, long n, int s, int *a, int *b, int *c)
{
    int i = (int)(n % g->nx), j = (int)((n / g->nx) % g->ny), k = (int)(n / ((long)g->nx * g->ny));
    *a = d->lo[0][i] + (s & 1);
    *b = d->lo[1][j] + ((s >> 1) & 1);
    *c = d->lo[2][k] + ((s >> 2) & 1);
    if (*a >= d->nb[0] || *b >= d->nb[1] || *c >= d->nb[2]) return -1;
    return (long)*a + (long)d->nb[0] * ((long)*b + (long)d->nb[1] * (long)*c);
}

int or_num_coarse(const og_grid *g)
{
    return or_num_blocks(g->nx, g->rx) * or_num_blocks(g->ny, g->ry) * or_num_blocks(g->nz, g->rz);
}

/* Dense solve M X = B (m x m, nrhs columns, row-major, both overwritten)
 * by Gaussian elimination with partial pivoting.  Returns 0 on success. */
static int dense_solve(int m, double *M, int nrhs, double *B)
{
    for (int k = 0; k < m; k++) {
        int p = k;
        for (int i = k + 1; i < m; i++)
            if (fabs(M[(long)i * m + k]) > fabs(M[(long)p * m + k])) p = i;
        if (M[(long)p * m + k] == 0.0) return -1;
        if (p != k) {
            for (int j = 0; j < m; j++) { double t = M[(long)k * m + j]; M[(long)k * m + j] = M[(long)p * m + j]; M[(long)p * m + j] = t; }
            for (int j = 0; j < nrhs; j++) { double t = B[(long)k * nrhs + j]; B[(long)k * nrhs + j] = B[(long)p * nrhs + j]; B[(long)p * nrhs + j] = t; }
        }
        for (int i = k + 1; i < m; i++) {
            double l = M[(long)i * m + k] / M[(long)k * m + k];
            if (l == 0.0) continue;
            for (int j = k; j < m; j++) M[(long)i * m + j] -= l * M[(long)k * m + j];
            for (int j = 0; j < nrhs; j++) B[(long)i * nrhs + j] -= l * B[(long)k * nrhs + j];
        }
    }
    for (int k = m - 1; k >= 0; k--)
        for (int j = 0; j < nrhs; j++) {
            double s = B[(long)k * nrhs + j];
            for (int c = k + 1; c < m; c++) s -= M[(long)k * m + c] * B[(long)c * nrhs + j];
            B[(long)k * nrhs + j] = s / M[(long)k * m + k];
        }
    return 0;
}

/* ------------------------------------------------------------------------
 * Basis functions of type B4 (Sec. 3, Eq. (11): -div(lambda grad Phi) = 0)
 * with reduced-problem boundary conditions on the dual-coarse cells.
 * Operator: the incompressible two-point matrix T (T_ii = sum_j T_ij,
 * T_ij = -T_ij; no density, accumulation or wells).
 *
 * Vertices carry the unit value of their own coarse node.  Then, level by
 * level downward (edges, faces, interiors), each connected set of
 * same-level cells (a dual edge segment, face patch or interior box) is
 * solved as one local problem:
 *   M_ii = sum of T_ij over neighbours j of the same or a higher level
 *          (couplings to lower levels are lumped away),
 *   M_ij = -T_ij for same-level neighbours,
 *   rhs_i,k = sum of T_ij Phi_jk over higher-level neighbours j,
 * with a dense direct solve.  Phi is stored per cell as 8 slot weights
 * (slot = position of the node among the bracketing vertices), slot-major:
 * P[s*N + n].  `only_region_cell` >= 0 restricts the work to the regions
 * needed for that cell (used to sample large grids); pass -1 for all.
 * Returns 0, or -1 if a local system is singular or a node falls outside
 * the bracketing vertices.
 * Pinned: partition of unity, 0 <= Phi <= 1, unit value at own vertex,
 * bilinear/trilinear hat for homogeneous k, series-resistance edges.
 * ---------------------------------------------------------------------- */
/* Local problem of one dual region (the connected set of cells of level L
 * given in `rc_cells`): unknowns are its cells, Dirichlet data the basis
 * values already set on higher-level neighbours, couplings to lower-level
 * neighbours lumped (left out of the row).  Writes the region's basis
 * values into P.  `pos` is scratch of N entries, -1 outside the call for
 * the region's cells.  Returns 0, or -1 if the local matrix is singular or
 * a value falls on a node that does not bracket its cell. */
static int solve_region(const og_grid *g, const og_dual *dd, const double *Tx, const double *Ty,
                        const double *Tz, const double *adiag, const int *level, long *pos,
                        const long *rc_cells, long m, int L, long N, double *P)
{
    og_dual d = *dd;
    int rc = 0;
    for (long a = 0; a < m; a++) pos[rc_cells[a]] = a;
    /* coarse nodes reached through higher-level neighbours */
    long nodes[64]; int nn = 0;
    for (long a = 0; a < m; a++) {
        long n = rc_cells[a];
        for (int fc = 0; fc < 6; fc++) {
            long nb; double T;
            if (!neighbour(g, Tx, Ty, Tz, n, fc, &nb, &T)) continue;
            if (level[nb] <= L) continue;
            for (int s = 0; s < 8; s++) {
                if (P[(long)s * N + nb] == 0.0) continue;
                int ia, ib, ic;
                long node = node_of_slot(g, &d, nb, s, &ia, &ib, &ic);
                int seen = 0;
                for (int t = 0; t < nn; t++) if (nodes[t] == node) seen = 1;
                if (!seen && nn < 64) nodes[nn++] = node;
            }
        }
    }
    double *M = (double *)calloc((size_t)m * m, sizeof(double));
    double *B = (double *)calloc((size_t)m * (nn > 0 ? nn : 1), sizeof(double));
    for (long a = 0; a < m; a++) {
        long n = rc_cells[a];
        if (adiag) M[a * m + a] += adiag[n];       /* accumulation term of B1 / B3 */
        for (int fc = 0; fc < 6; fc++) {
            long nb; double T;
            if (!neighbour(g, Tx, Ty, Tz, n, fc, &nb, &T)) continue;
            if (level[nb] < L) continue;             /* lumped */
            M[a * m + a] += T;
            if (level[nb] == L) { M[a * m + pos[nb]] -= T; continue; }
            for (int s = 0; s < 8; s++) {
                double w = P[(long)s * N + nb];
                if (w == 0.0) continue;
                int ia, ib, ic;
                long node = node_of_slot(g, &d, nb, s, &ia, &ib, &ic);
                for (int t = 0; t < nn; t++) if (nodes[t] == node) B[a * nn + t] += T * w;
            }
        }
    }
    if (nn > 0 && dense_solve((int)m, M, nn, B) != 0) rc = -1;
    for (long a = 0; a < m && rc == 0; a++) {
        long n = rc_cells[a];
        for (int t = 0; t < nn; t++) {
            long node = nodes[t];
            int ia = (int)(node % d.nb[0]), ib = (int)((node / d.nb[0]) % d.nb[1]), ic = (int)(node / ((long)d.nb[0] * d.nb[1]));
            int s = node_slot(g, &d, n, ia, ib, ic);
            if (s < 0) { if (B[a * nn + t] != 0.0) rc = -1; continue; }
            P[(long)s * N + n] = B[a * nn + t];
        }
    }
    for (long a = 0; a < m; a++) pos[rc_cells[a]] = -1;
    free(M); free(B);
    return rc;
}

/* Basis of a general local operator (Sec. 3, Eqs. (8)-(11)): face
 * couplings Cx/Cy/Cz (T for B3/B4, the density-weighted W = T rho_f of the
 * current iterate for B1/B2) and an optional extra diagonal adiag (the
 * accumulation term of B1/B3; NULL for B2/B4).  Same wirebasket order and
 * reduced boundary conditions as B4. */
int or_basis_general(const og_grid *g, const double *Tx, const double *Ty, const double *Tz,
                     const double *adiag, double *P);

int or_basis_b4(const og_grid *g, const double *Tx, const double *Ty, const double *Tz,
                double *P)
{
    return or_basis_general(g, Tx, Ty, Tz, NULL, P);
}

int or_basis_general(const og_grid *g, const double *Tx, const double *Ty, const double *Tz,
                     const double *adiag, double *P)
{
    long N = ncells(g);
    og_dual d; dual_init(g, &d);
    int *level = (int *)malloc(sizeof(int) * N);
    long *region = (long *)malloc(sizeof(long) * N);
    long *stack = (long *)malloc(sizeof(long) * N);
    long *cells = (long *)malloc(sizeof(long) * N);
    long *pos = (long *)malloc(sizeof(long) * N);
    int rc = 0;
    for (long n = 0; n < N; n++) { level[n] = cell_level(g, &d, n); region[n] = -1; pos[n] = -1; }
    memset(P, 0, sizeof(double) * 8 * N);
    for (long n = 0; n < N; n++)
        if (level[n] == d.dim) P[0 * N + n] = 1.0;   /* own node sits in slot 0 */

    long *rstart = (long *)malloc(sizeof(long) * (N + 1));
    for (int L = d.dim - 1; L >= 0 && rc == 0; L--) {
        /* the connected sets (regions) of level-L cells, by flood fill; the
         * cells of region q are cells[rstart[q] .. rstart[q+1]) */
        long nreg = 0, m = 0;
        for (long seed = 0; seed < N; seed++) {
            if (level[seed] != L || region[seed] >= 0) continue;
            long top = 0;
            rstart[nreg++] = m;
            stack[top++] = seed; region[seed] = seed;
            while (top > 0) {
                long n = stack[--top];
                cells[m++] = n;
                for (int fc = 0; fc < 6; fc++) {
                    long nb; double T;
                    if (!neighbour(g, Tx, Ty, Tz, n, fc, &nb, &T)) continue;
                    if (level[nb] == L && region[nb] < 0) { region[nb] = seed; stack[top++] = nb; }
                }
            }
        }
        rstart[nreg] = m;
        /* one local problem per region; regions of a level only read basis
         * values of higher levels, so they are independent */
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rc)
        for (long q = 0; q < nreg; q++) {
            const long *rc_cells = cells + rstart[q];
            long mq = rstart[q + 1] - rstart[q];
            if (solve_region(g, &d, Tx, Ty, Tz, adiag, level, pos, rc_cells, mq, L, N, P) != 0) rc |= 1;
        }
    }
    if (rc) rc = -1;
    free(rstart);
    free(level); free(region); free(stack); free(cells); free(pos);
    dual_free(&d);
    return rc;
}

/* Coarse node index of slot s of cell n, or -1 (for the Python side). */
void or_slot_nodes(const og_grid *g, int32_t *node)
{
    og_dual d; dual_init(g, &d);
    long N = ncells(g);
    for (long n = 0; n < N; n++)
        for (int s = 0; s < 8; s++) {
            int a, b, c;
            node[(long)s * N + n] = (int32_t)node_of_slot(g, &d, n, s, &a, &b, &c);
        }
    dual_free(&d);
}

/* Primal block (coarse node) containing each cell. */
void or_primal_block(const og_grid *g, int32_t *blk)
{
    int nbx = or_num_blocks(g->nx, g->rx), nby = or_num_blocks(g->ny, g->ry);
    for (int k = 0; k < g->nz; k++)
        for (int j = 0; j < g->ny; j++)
            for (int i = 0; i < g->nx; i++)
                blk[cell_index(g, i, j, k)] = (i / g->rx) + nbx * ((j / g->ry) + nby * (k / g->rz));
}

/* ------------------------------------------------------------------------
 * Coarse operator (Sec. 3, Eq. (13)):  A_c = R A P_hat, with P_hat the basis
 * with Dirichlet rows zeroed and R = R^FV (Eq. (7): 0/1 sums over primal
 * blocks) or R^FE = P_hat^T.  Dense, row-major Nc x Nc.
 * Pinned: explicit sparse triple product; MSFE symmetry/SPD.
 * ---------------------------------------------------------------------- */
void or_coarse_operator(const og_grid *g, const double *Wx, const double *Wy, const double *Wz,
                        const double *diag, const uint8_t *dmask, const double *P,
                        int restriction, double *Ac)
{
    og_dual d; dual_init(g, &d);
    long N = ncells(g);
    int Nc = or_num_coarse(g);
    int32_t *blk = (int32_t *)malloc(sizeof(int32_t) * N);
    or_primal_block(g, blk);
    memset(Ac, 0, sizeof(double) * (size_t)Nc * Nc);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; n++) {
        long ids[64]; double vals[64];
        int cnt = 0;
        /* row n of A P_hat as a short list of (coarse node, value) */
        for (int fc = -1; fc < 6; fc++) {
            long m = n; double coef = diag[n];
            if (fc >= 0) {
                double W;
                if (!neighbour(g, Wx, Wy, Wz, n, fc, &m, &W)) continue;
                coef = -W;
            }
            if (dmask[m]) continue;
            for (int s = 0; s < 8; s++) {
                double w = P[(long)s * N + m];
                if (w == 0.0) continue;
                int a, b, c;
                long node = node_of_slot(g, &d, m, s, &a, &b, &c);
                int t = 0;
                while (t < cnt && ids[t] != node) t++;
                if (t == cnt) { ids[cnt] = node; vals[cnt] = 0.0; cnt++; }
                vals[t] += coef * w;
            }
        }
        if (restriction == OR_FV) {
            for (int t = 0; t < cnt; t++) {
#pragma omp atomic
                Ac[(long)blk[n] * Nc + ids[t]] += vals[t];
            }
        } else {
            if (dmask[n]) continue;
            for (int s = 0; s < 8; s++) {
                double w = P[(long)s * N + n];
                if (w == 0.0) continue;
                int a, b, c;
                long k = node_of_slot(g, &d, n, s, &a, &b, &c);
                for (int t = 0; t < cnt; t++) {
#pragma omp atomic
                    Ac[k * Nc + ids[t]] += w * vals[t];
                }
            }
        }
    }
    free(blk);
    dual_free(&d);
}

/* Restriction of a fine vector: FV block sums (Eq. (7)) or P_hat^T x. */
void or_restrict(const og_grid *g, const uint8_t *dmask, const double *P, int restriction,
                 const double *x, double *xc)
{
    og_dual d; dual_init(g, &d);
    long N = ncells(g);
    int Nc = or_num_coarse(g);
    memset(xc, 0, sizeof(double) * Nc);
    if (restriction == OR_FV) {
        int32_t *blk = (int32_t *)malloc(sizeof(int32_t) * N);
        or_primal_block(g, blk);
        for (long n = 0; n < N; n++) xc[blk[n]] += x[n];
        free(blk);
    } else {
#pragma omp parallel for schedule(static)
        for (long n = 0; n < N; n++) {
            if (dmask[n]) continue;
            for (int s = 0; s < 8; s++) {
                double w = P[(long)s * N + n];
                if (w == 0.0) continue;
                int a, b, c;
                long k = node_of_slot(g, &d, n, s, &a, &b, &c);
#pragma omp atomic
                xc[k] += w * x[n];
            }
        }
    }
    dual_free(&d);
}

/* Prolongation (Sec. 3, Eq. (12)): x = P_hat xc. */
void or_prolong(const og_grid *g, const uint8_t *dmask, const double *P, const double *xc, double *x)
{
    og_dual d; dual_init(g, &d);
    long N = ncells(g);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; n++) {
        double s = 0.0;
        if (!dmask[n])
            for (int t = 0; t < 8; t++) {
                double w = P[(long)t * N + n];
                if (w == 0.0) continue;
                int a, b, c;
                long k = node_of_slot(g, &d, n, t, &a, &b, &c);
                s += w * xc[k];
            }
        x[n] = s;
    }
    dual_free(&d);
}

/* ------------------------------------------------------------------------
 * Coarse solve (Sec. 3, Eq. (15)): LU factorisation with partial pivoting
 * (Doolittle, row-major, in place) and the corresponding solve.
 * Pinned: numpy.linalg.solve.
 * ---------------------------------------------------------------------- */
int or_lu_factor(int n, double *A, int32_t *piv)
{
    for (int k = 0; k < n; k++) {
        int p = k;
        for (int i = k + 1; i < n; i++)
            if (fabs(A[(long)i * n + k]) > fabs(A[(long)p * n + k])) p = i;
        piv[k] = p;
        if (A[(long)p * n + k] == 0.0) return -1;
        if (p != k)
            for (int j = 0; j < n; j++) { double t = A[(long)k * n + j]; A[(long)k * n + j] = A[(long)p * n + j]; A[(long)p * n + j] = t; }
#pragma omp parallel for schedule(static) if (n - k > 64)
        for (int i = k + 1; i < n; i++) {
            A[(long)i * n + k] /= A[(long)k * n + k];
            double l = A[(long)i * n + k];
            for (int j = k + 1; j < n; j++) A[(long)i * n + j] -= l * A[(long)k * n + j];
        }
    }
    return 0;
}

void or_lu_solve(int n, const double *LU, const int32_t *piv, double *b)
{
    for (int k = 0; k < n; k++)
        if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < i; j++) b[i] -= LU[(long)i * n + j] * b[j];
    for (int i = n - 1; i >= 0; i--) {
        for (int j = i + 1; j < n; j++) b[i] -= LU[(long)i * n + j] * b[j];
        b[i] /= LU[(long)i * n + i];
    }
}

/* ------------------------------------------------------------------------
 * ILU(0) smoother (Sec. 3, Table "cams" step 6; the paper cites Saad's
 * textbook for ILU(0)).  Generic incomplete LU with zero fill of the
 * matrix permuted to a given ordering, on a CSR copy of the 7-point
 * operator; `order[t]` is the cell placed at position t.
 * Two orderings are used: natural (order = identity) and red-black (cells
 * with even i+j+k first, each colour in natural order).
 * Pinned: (L U)_ij = A_ij on the sparsity pattern; apply = explicit
 * triangular solves.
 * ---------------------------------------------------------------------- */
typedef struct {
    long n;
    long *rowptr;
    long *col;      /* positions (permuted indices), sorted per row */
    double *val;
    long *diagpos;
    long *order;    /* position -> cell */
    long *where;    /* cell -> position */
    long nblk;      /* block-Jacobi factors: independent blocks (0 otherwise) */
    long *blkptr;   /* positions of block b: blkpos[blkptr[b] .. blkptr[b+1]), ascending */
    long *blkpos;
} og_ilu;

void *or_ilu0_create(const og_grid *g, const double *Wx, const double *Wy, const double *Wz,
                     const double *diag, const int64_t *order)
{
    og_ilu *M = (og_ilu *)calloc(1, sizeof(og_ilu));
    long N = ncells(g);
    M->n = N;
    M->order = (long *)malloc(sizeof(long) * N);
    M->where = (long *)malloc(sizeof(long) * N);
    for (long t = 0; t < N; t++) { M->order[t] = (long)order[t]; M->where[order[t]] = t; }
    M->rowptr = (long *)malloc(sizeof(long) * (N + 1));
    M->col = (long *)malloc(sizeof(long) * 7 * N);
    M->val = (double *)malloc(sizeof(double) * 7 * N);
    M->diagpos = (long *)malloc(sizeof(long) * N);
    long nnz = 0;
    for (long t = 0; t < N; t++) {
        long n = M->order[t];
        M->rowptr[t] = nnz;
        long cs[7]; double vs[7]; int c = 0;
        cs[c] = t; vs[c] = diag[n]; c++;
        for (int fc = 0; fc < 6; fc++) {
            long m; double W;
            if (!neighbour(g, Wx, Wy, Wz, n, fc, &m, &W)) continue;
            if (W == 0.0) continue;
            cs[c] = M->where[m]; vs[c] = -W; c++;
        }
        /* insertion sort by column */
        for (int a = 1; a < c; a++)
            for (int b = a; b > 0 && cs[b - 1] > cs[b]; b--) {
                long tc = cs[b]; cs[b] = cs[b - 1]; cs[b - 1] = tc;
                double tv = vs[b]; vs[b] = vs[b - 1]; vs[b - 1] = tv;
            }
        for (int a = 0; a < c; a++) {
            M->col[nnz] = cs[a]; M->val[nnz] = vs[a];
            if (cs[a] == t) M->diagpos[t] = nnz;
            nnz++;
        }
    }
    M->rowptr[N] = nnz;
    /* IKJ incomplete factorisation restricted to the pattern */
    for (long i = 1; i < N; i++) {
        for (long pk = M->rowptr[i]; pk < M->rowptr[i + 1] && M->col[pk] < i; pk++) {
            long k = M->col[pk];
            M->val[pk] /= M->val[M->diagpos[k]];
            double lik = M->val[pk];
            for (long pj = pk + 1; pj < M->rowptr[i + 1]; pj++) {
                long j = M->col[pj];
                for (long q = M->rowptr[k]; q < M->rowptr[k + 1]; q++)
                    if (M->col[q] == j) { M->val[pj] -= lik * M->val[q]; break; }
            }
        }
    }
    return M;
}

void or_ilu0_free(void *h)
{
    og_ilu *M = (og_ilu *)h;
    if (!M) return;
    free(M->rowptr); free(M->col); free(M->val); free(M->diagpos); free(M->order); free(M->where);
    free(M->blkptr); free(M->blkpos);
    free(M);
}

/* Export the factor (positions, values) for the pins. */
long or_ilu0_nnz(void *h) { return ((og_ilu *)h)->rowptr[((og_ilu *)h)->n]; }

void or_ilu0_export(void *h, int64_t *rowptr, int64_t *col, double *val)
{
    og_ilu *M = (og_ilu *)h;
    for (long t = 0; t <= M->n; t++) rowptr[t] = M->rowptr[t];
    for (long q = 0; q < M->rowptr[M->n]; q++) { col[q] = M->col[q]; val[q] = M->val[q]; }
}

/* x = (L U)^{-1} z, in cell order.  A block-Jacobi factor has no coupling
 * between its blocks, so each block's triangular solves run on their own
 * (same operations per row as the whole-matrix sweep). */
void or_ilu0_apply(void *h, const double *z, double *x)
{
    og_ilu *M = (og_ilu *)h;
    long N = M->n;
    double *y = (double *)malloc(sizeof(double) * N);
    if (M->nblk > 0) {
#pragma omp parallel for schedule(static)
        for (long b = 0; b < M->nblk; b++) {
            for (long u = M->blkptr[b]; u < M->blkptr[b + 1]; u++) {
                long t = M->blkpos[u];
                double s = z[M->order[t]];
                for (long q = M->rowptr[t]; q < M->diagpos[t]; q++) s -= M->val[q] * y[M->col[q]];
                y[t] = s;
            }
            for (long u = M->blkptr[b + 1] - 1; u >= M->blkptr[b]; u--) {
                long t = M->blkpos[u];
                double s = y[t];
                for (long q = M->diagpos[t] + 1; q < M->rowptr[t + 1]; q++) s -= M->val[q] * y[M->col[q]];
                y[t] = s / M->val[M->diagpos[t]];
            }
        }
        for (long t = 0; t < N; t++) x[M->order[t]] = y[t];
        free(y);
        return;
    }
    for (long t = 0; t < N; t++) {
        double s = z[M->order[t]];
        for (long q = M->rowptr[t]; q < M->diagpos[t]; q++) s -= M->val[q] * y[M->col[q]];
        y[t] = s;
    }
    for (long t = N - 1; t >= 0; t--) {
        double s = y[t];
        for (long q = M->diagpos[t] + 1; q < M->rowptr[t + 1]; q++) s -= M->val[q] * y[M->col[q]];
        y[t] = s / M->val[M->diagpos[t]];
    }
    for (long t = 0; t < N; t++) x[M->order[t]] = y[t];
    free(y);
}

/* Block-Jacobi ILU(0): the couplings across the faces of bx x by x bz cell
 * blocks are removed, and ILU(0) in natural order is taken of what remains;
 * the blocks are then independent of each other.  The smoothing residual
 * still uses the full matrix.  Blocks are aligned at the origin (the last
 * block of an axis possibly shorter), or, with offsets (ox, oy, oz), laid on
 * the axis shifted cyclically: along x, cell i sits at position
 * (i + ox) mod nx and the block holds 8 consecutive positions, so the first
 * block may consist of a piece at the far end of the axis and a piece at
 * its start (the two pieces share no coupling, so their ILU(0) factors are
 * independent).  Two cells of a row are coupled in the factor iff their
 * positions fall in the same block; an axis of at most b cells is then one
 * block for any offset. */
static int same_block(int i, int n, int b, int o)
{
    return ((i + o) % n) / b == ((i + 1 + o) % n) / b;
}

void *or_ilu0_block_create_shifted(const og_grid *g, const double *Wx, const double *Wy, const double *Wz,
                                   const double *diag, int bx, int by, int bz, int ox, int oy, int oz)
{
    long N = ncells(g);
    double *W = (double *)malloc(sizeof(double) * 3 * N);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * N);
    for (int k = 0; k < g->nz; k++)
        for (int j = 0; j < g->ny; j++)
            for (int i = 0; i < g->nx; i++) {
                long n = cell_index(g, i, j, k);
                W[n] = same_block(i, g->nx, bx, ox) ? Wx[n] : 0.0;
                W[N + n] = same_block(j, g->ny, by, oy) ? Wy[n] : 0.0;
                W[2 * N + n] = same_block(k, g->nz, bz, oz) ? Wz[n] : 0.0;
                order[n] = n;
            }
    og_ilu *M = (og_ilu *)or_ilu0_create(g, W, W + N, W + 2 * N, diag, order);
    free(W);
    free(order);
    /* block lists (natural order = positions) */
    int nb[3] = {(g->nx + bx - 1) / bx, (g->ny + by - 1) / by, (g->nz + bz - 1) / bz};
    M->nblk = (long)nb[0] * nb[1] * nb[2];
    M->blkptr = (long *)calloc(M->nblk + 1, sizeof(long));
    M->blkpos = (long *)malloc(sizeof(long) * N);
    long *id = (long *)malloc(sizeof(long) * N);
    for (int k = 0; k < g->nz; k++)
        for (int j = 0; j < g->ny; j++)
            for (int i = 0; i < g->nx; i++) {
                long n = cell_index(g, i, j, k);
                id[n] = ((i + ox) % g->nx) / bx + (long)nb[0] * (((j + oy) % g->ny) / by + (long)nb[1] * (((k + oz) % g->nz) / bz));
                M->blkptr[id[n] + 1]++;
            }
    for (long b = 0; b < M->nblk; b++) M->blkptr[b + 1] += M->blkptr[b];
    long *fill = (long *)malloc(sizeof(long) * M->nblk);
    for (long b = 0; b < M->nblk; b++) fill[b] = M->blkptr[b];
    for (long n = 0; n < N; n++) M->blkpos[fill[id[n]]++] = n;
    free(fill);
    free(id);
    return M;
}

void *or_ilu0_block_create(const og_grid *g, const double *Wx, const double *Wy, const double *Wz,
                           const double *diag, int bx, int by, int bz)
{
    return or_ilu0_block_create_shifted(g, Wx, Wy, Wz, diag, bx, by, bz, 0, 0, 0);
}

/* The red-black ordering used by the smoother. */
void or_redblack_order(const og_grid *g, int64_t *order)
{
    long t = 0;
    for (int colour = 0; colour < 2; colour++)
        for (int k = 0; k < g->nz; k++)
            for (int j = 0; j < g->ny; j++)
                for (int i = 0; i < g->nx; i++)
                    if (((i + j + k) & 1) == colour) order[t++] = cell_index(g, i, j, k);
}

/* ------------------------------------------------------------------------
 * C-AMS iteration (Sec. 3, Table "cams"; Eqs. (12)-(15)), without
 * correction functions, solving A d = r0 for the Newton update d:
 *   repeat:  r = r0 - A d;  stop when ||r|| <= rtol ||r0||;
 *            n_pre ILU(0) Richardson steps on A e = r  (d += e, r -= A e);
 *            d1 = P_hat A_c^{-1} R r;  d += d1;  r1 = r - A d1;
 *            d2 = 0; n_post times: d2 += M^{-1}(r1 - A d2);  d += d2.
 * With a second smoother `ilu_alt` (nullable) the Richardson steps of each
 * smoothing stage take M = ilu, ilu_alt, ilu, ... (the first step of the
 * stage takes ilu).
 * Stops when ||r|| <= rtol ||r0|| or ||r|| <= atol (atol = 0: relative only).
 * Returns the number of iterations (>= 0), or -1 if maxit was reached;
 * hist (length maxit+1, nullable) receives ||r||/||r0|| per iteration.
 * Pinned: MSFV zero block residual / MSFE Galerkin orthogonality after the
 * coarse stage; convergence to the sparse direct solution.
 * ---------------------------------------------------------------------- */
int or_cams_solve(const og_grid *g, const double *Wx, const double *Wy, const double *Wz,
                  const double *diag, const uint8_t *dmask, const double *P, int restriction,
                  const double *LU, const int32_t *piv, void *ilu, void *ilu_alt,
                  int n_pre, int n_post, double rtol, double atol, int maxit,
                  const double *r0, double *dsol, double *hist)
{
    long N = ncells(g);
    int Nc = or_num_coarse(g);
    double *r = (double *)malloc(sizeof(double) * N);
    double *t = (double *)malloc(sizeof(double) * N);
    double *e = (double *)malloc(sizeof(double) * N);
    double *x = (double *)malloc(sizeof(double) * N);
    double *rc = (double *)malloc(sizeof(double) * Nc);
    double nr0 = 0.0;
    for (long n = 0; n < N; n++) { dsol[n] = 0.0; nr0 += r0[n] * r0[n]; }
    nr0 = sqrt(nr0);
    int it = 0, result = -1;
    for (;; it++) {
        or_matvec(g, Wx, Wy, Wz, diag, dsol, t);
        double nr = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : nr)
        for (long n = 0; n < N; n++) { r[n] = r0[n] - t[n]; nr += r[n] * r[n]; }
        nr = sqrt(nr);
        double rel = nr0 > 0 ? nr / nr0 : 0.0;
        if (hist && it <= maxit) hist[it] = rel;
        if (rel <= rtol || nr <= atol || nr0 == 0.0) { result = it; break; }
        if (it >= maxit || !isfinite(rel)) break;
        /* optional pre-smoothing */
        if (n_pre > 0) {
            #pragma omp parallel for schedule(static)
            for (long n = 0; n < N; n++) e[n] = 0.0;
            for (int s = 0; s < n_pre; s++) {
                or_matvec(g, Wx, Wy, Wz, diag, e, t);
                #pragma omp parallel for schedule(static)
                for (long n = 0; n < N; n++) t[n] = r[n] - t[n];
                or_ilu0_apply((s & 1) && ilu_alt ? ilu_alt : ilu, t, x);
                #pragma omp parallel for schedule(static)
                for (long n = 0; n < N; n++) e[n] += x[n];
            }
            or_matvec(g, Wx, Wy, Wz, diag, e, t);
            #pragma omp parallel for schedule(static)
            for (long n = 0; n < N; n++) { dsol[n] += e[n]; r[n] -= t[n]; }
        }
        /* multiscale stage, Eq. (15) */
        or_restrict(g, dmask, P, restriction, r, rc);
        or_lu_solve(Nc, LU, piv, rc);
        or_prolong(g, dmask, P, rc, e);
        or_matvec(g, Wx, Wy, Wz, diag, e, t);
        #pragma omp parallel for schedule(static)
        for (long n = 0; n < N; n++) { dsol[n] += e[n]; r[n] -= t[n]; }
        /* post-smoothing on r1 = r - A d1 */
        #pragma omp parallel for schedule(static)
        for (long n = 0; n < N; n++) e[n] = 0.0;
        for (int s = 0; s < n_post; s++) {
            or_matvec(g, Wx, Wy, Wz, diag, e, t);
            #pragma omp parallel for schedule(static)
            for (long n = 0; n < N; n++) t[n] = r[n] - t[n];
            or_ilu0_apply((s & 1) && ilu_alt ? ilu_alt : ilu, t, x);
            #pragma omp parallel for schedule(static)
            for (long n = 0; n < N; n++) e[n] += x[n];
        }
        #pragma omp parallel for schedule(static)
        for (long n = 0; n < N; n++) dsol[n] += e[n];
    }
    free(r); free(t); free(e); free(x); free(rc);
    return result;
}

/* ------------------------------------------------------------------------
 * One backward-Euler time step by the paper's Newton-Raphson linearisation
 * (Sec. 2; Table "cams" outer loop; Sec. 4.1.1 for the error norm):
 *   repeat: assemble A, r at p; if ||eps||_2 <= newton_tol stop;
 *           coarse operator + LU; ILU(0) smoother (smoother 0: red-black
 *           order; 1: block-Jacobi ILU(0) on bx x by x bz blocks; 2: the
 *           same blocks alternating, step by step, with the block grid
 *           shifted cyclically by half a block, (bx/2, by/2, bz/2); 3: the
 *           whole matrix in natural order, the paper's global ILU(0)); C-AMS
 *           solve; p += d.
 * The basis P (type B4) is pressure independent and passed in.
 * stats[0] = Newton iterations, stats[1] = total linear iterations,
 * stats[2] = final ||eps||_2.  Returns 0, -1 (Newton not converged),
 * -2 (linear solve not converged) or -3 (singular coarse matrix).
 * ---------------------------------------------------------------------- */
int or_newton_step(const og_grid *g, const og_fluid *f,
                   const double *Tx, const double *Ty, const double *Tz,
                   const double *phi, const double *q, const uint8_t *dmask, const double *bt,
                   const double *bp, const double *P,
                   int restriction, int n_pre, int n_post, double lin_rtol, double lin_atol, int lin_maxit,
                   double newton_tol, int newton_maxit, int smoother, int bx, int by, int bz,
                   const double *pn, double *p, double *stats)
{
    long N = ncells(g);
    int Nc = or_num_coarse(g);
    double *W = (double *)malloc(sizeof(double) * 3 * N);
    double *diag = (double *)malloc(sizeof(double) * N);
    double *r = (double *)malloc(sizeof(double) * N);
    double *d = (double *)malloc(sizeof(double) * N);
    double *Ac = (double *)malloc(sizeof(double) * (size_t)Nc * Nc);
    int32_t *piv = (int32_t *)malloc(sizeof(int32_t) * Nc);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * N);
    if (smoother == 3)
        for (long n = 0; n < N; n++) order[n] = n;
    else
        or_redblack_order(g, order);
    int rc = -1, nit = 0, lit = 0;
    double en = 0.0;
    for (nit = 0; nit <= newton_maxit; nit++) {
        en = or_linear_system(g, f, Tx, Ty, Tz, phi, q, dmask, bt, bp, p, pn, W, W + N, W + 2 * N, diag, r);
        if (en <= newton_tol) { rc = 0; break; }
        if (nit == newton_maxit || !isfinite(en)) break;
        or_coarse_operator(g, W, W + N, W + 2 * N, diag, dmask, P, restriction, Ac);
        if (or_lu_factor(Nc, Ac, piv) != 0) { rc = -3; break; }
        void *ilu = (smoother == 1 || smoother == 2) ? or_ilu0_block_create(g, W, W + N, W + 2 * N, diag, bx, by, bz)
                                  : or_ilu0_create(g, W, W + N, W + 2 * N, diag, order);
        void *alt = smoother == 2 ? or_ilu0_block_create_shifted(g, W, W + N, W + 2 * N, diag, bx, by, bz,
                                                                 bx / 2, by / 2, bz / 2)
                                  : NULL;
        int its = or_cams_solve(g, W, W + N, W + 2 * N, diag, dmask, P, restriction, Ac, piv, ilu, alt,
                                n_pre, n_post, lin_rtol, lin_atol, lin_maxit, r, d, NULL);
        or_ilu0_free(ilu);
        or_ilu0_free(alt);
        if (its < 0) { rc = -2; lit += lin_maxit; break; }
        lit += its;
        for (long n = 0; n < N; n++) p[n] += d[n];
    }
    if (stats) { stats[0] = nit; stats[1] = lit; stats[2] = en; }
    free(W); free(diag); free(r); free(d); free(Ac); free(piv); free(order);
    return rc;
}
