/*
 * helm_oracle.h -- plain, slow, FP64 CPU oracle of the block shifted-Laplacian
 * multigrid / block FGMRES Helmholtz solve.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, includes or
 * calls this code; only the tests, the smoke check and the benchmark's CPU
 * baseline do. It shares no code, header, table or helper with the HIP path.
 *
 * Every routine follows a definition of the paper (Treister & Haber,
 * "Full waveform inversion guided by travel time tomography"):
 *   - operator: the discrete Helmholtz equation (eq:helm) discretised by
 *     second-order finite differences into A(m,omega)u = q (eq:LinearSystem),
 *     written here as H u = q with H = -Lap_h - omega^2 diag(m (1 - i gamma))
 *     (gamma dimensionless, the paper's gamma/omega; q negated);
 *   - shifted operator: the same with a positive constant beta added to gamma
 *     (section "Solving the Helmholtz equation for multiple right hand
 *     sides"; beta = 0.2 in the experiments of section 5.3);
 *   - transfers: bilinear/trilinear prolongation P and full weighting
 *     R = 2^-d P^T (same section);
 *   - Galerkin coarse operators A_c = R A P (the two-grid cycle text);
 *   - damped Jacobi relaxation, weight 0.8, 2 pre + 2 post (section 5.3);
 *   - two-grid cycle applied recursively = V-cycle (Algorithm "Two-grid
 *     cycle"); LU solve on the coarsest grid for a block of right-hand sides;
 *   - block FGMRES(m) preconditioned by the cycle (section 5.3).
 *
 * Conventions: complex numbers are C99 double _Complex (interleaved re, im).
 * A grid has nu[a] = n[a]-1 unknowns per axis, axis 0 fastest; for dim 2,
 * nu[2] = 1. Blocks of right-hand sides are [nrhs][N], each RHS contiguous.
 * Stencils are [N][27]: entry o = (ox+1) + 3(oy+1) + 9(oz+1) couples node i
 * to node i + (ox, oy, oz); in 2D only oz = 0 is used.
 */
#ifndef HELM_ORACLE_H
#define HELM_ORACLE_H

#include <complex.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef double _Complex ozc;

typedef struct {
  int dim;
  int nu[3];    /* unknowns per axis, axis 0 fastest; nu[2] = 1 in 2D */
  double h[3];  /* spacing per axis */
} og_grid;

int64_t og_npts(const og_grid* g);
/* Grid of the next coarser level: half the cells, twice the spacing. */
void og_coarsen(const og_grid* f, og_grid* c);

/* out = (-Lap_h - omega^2 m (1 - i(gamma + beta))) u, Dirichlet outside. */
void orc_apply_fine(const og_grid* g, const double* m, const double* gamma,
                    double omega, double beta, int nrhs, const ozc* u, ozc* out);
/* The same operator written as a 27-entry stencil per node. */
void orc_fine_stencil(const og_grid* g, const double* m, const double* gamma,
                      double omega, double beta, ozc* st);
/* out = S u for a stencil operator. */
void orc_apply_stencil(const og_grid* g, const ozc* st, int nrhs, const ozc* u, ozc* out);
/* uf = P ec (overwrites uf); fine grid g, coarse grid og_coarsen(g). */
void orc_prolong(const og_grid* g, int nrhs, const ozc* ec, ozc* uf);
/* rc = 2^-d P^T rf. */
void orc_restrict(const og_grid* g, int nrhs, const ozc* rf, ozc* rc);
/* Galerkin coarse stencil R S P by probing with 3^d coloured unit vectors.
 * If stf == NULL the fine operator is the shifted fine operator (m, gamma,
 * omega, beta). */
void orc_galerkin(const og_grid* g, const ozc* stf, const double* m, const double* gamma,
                  double omega, double beta, ozc* stc);
/* nsweep damped-Jacobi sweeps u <- u + w D^-1 (f - S u), D = diag(S). */
void orc_jacobi(const og_grid* g, const ozc* st, double w, int nsweep, int nrhs,
                const ozc* f, ozc* u);

/* Banded LU with partial pivoting of a stencil operator in lexicographic order. */
typedef struct {
  int64_t n, kl, ku, ld;  /* order, lower/upper bandwidth, row storage width */
  ozc* a;                 /* n x ld: row i holds columns i-kl .. i-kl+ld-1 */
  int64_t* piv;
} orc_band;
int orc_band_factor(const og_grid* g, const ozc* st, orc_band* out);
void orc_band_solve(const orc_band* b, int nrhs, ozc* x);
void orc_band_free(orc_band* b);

/* Multigrid hierarchy of the shifted operator. The coarsest grid is solved
 * by LU (banded, partial pivoting), by coarse_iters steps of GMRES from zero
 * (an inexact iterative coarsest solve, as the paper discusses for large
 * coarse grids in section 5.3), or only relaxed. */
enum { ORC_COARSE_LU = 0, ORC_COARSE_GMRES = 1, ORC_COARSE_NONE = 2 };
typedef struct orc_hier orc_hier;
orc_hier* orc_setup(const og_grid* g, const double* m, const double* gamma, double omega,
                    double beta, int levels, const int* nu_pre, const int* nu_post,
                    const double* wjac, int coarse_kind, int coarse_iters);
void orc_free(orc_hier* H);
int orc_levels(const orc_hier* H);
void orc_level_grid(const orc_hier* H, int l, og_grid* g);
/* Copy out the Galerkin stencil of level l >= 1 ([N_l][27]). */
void orc_level_stencil(const orc_hier* H, int l, ozc* st);
/* u = V-cycle(f) for each RHS column (u is overwritten). */
void orc_vcycle(const orc_hier* H, int nrhs, const ozc* f, ozc* u);
/* The coarsest-grid solve as used inside the cycle (M_L^-1 f for LU). */
void orc_coarse_solve(const orc_hier* H, int nrhs, const ozc* f, ozc* u);
/* GMRES coarsest solve as `restarts` cycles of coarse_iters steps (restarted
 * GMRES; the default is one cycle). */
void orc_set_coarse_restarts(orc_hier* H, int restarts);
/* 1: W-cycle. The coarse problem of every level whose coarse level is not
 * the coarsest gets two cycles, the second on the residual of the first
 * (e_c += B_c(r_c - M_c e_c)); the coarsest level is solved once. 0: V. */
void orc_set_cycle_w(orc_hier* H, int w);
/* 1: K-cycle (the paper's K-FGMRES): every coarse level but the coarsest is
 * solved by two flexible GMRES steps from zero, each preconditioned by that
 * level's cycle. 0: V. */
void orc_set_cycle_k(orc_hier* H, int k);

/* Block FGMRES(restart) for H X = Q with X0 = 0 (or X on entry if warm).
 * Right preconditioning by the V-cycle (or identity if H == NULL-prec flag).
 * Stops when every column has ||q_s - H x_s|| / ||q_s|| <= tol (FP64 true
 * residual) or after maxit preconditioner applications.
 * Returns 0 if converged, 1 otherwise. iters = preconditioned Arnoldi steps
 * (the paper's cycle count); relres[p] = final true relative residuals;
 * hist (optional, length maxit): max-over-columns estimated relres per step. */
int orc_block_fgmres(const orc_hier* H, int use_prec, int p, const ozc* Q, ozc* X,
                     int warm, double tol, int restart, int maxit, int* iters,
                     double* relres, double* hist);

/* Small dense helpers (exported for their pins). */
/* Householder QR of an N x p column-major complex matrix: A is replaced by Q
 * (N x p, orthonormal columns), R (p x p, column-major upper) written out. */
void orc_householder_qr(int64_t N, int p, ozc* A, ozc* R);
/* Rank-revealing Householder QR with column pivoting (stops at a remaining
 * column norm <= tol * largest column norm): A becomes Q (zero columns past
 * the rank), R (p x p, column-major) the factor in the original column order
 * with zero rows past the rank. Returns the rank. */
int orc_householder_qr_rr(int64_t N, int p, ozc* A, ozc* R, double tol);
/* min ||B - A Y||_F with A m x n (m >= n, full rank apart from columns of
 * zeros, whose coefficients are 0), B m x k, column-major.
 * Y (n x k) written out; res (k) = column norms of the residual. */
void orc_lstsq(int mrows, int ncols, int k, const ozc* A, const ozc* B, ozc* Y, double* res);

int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
