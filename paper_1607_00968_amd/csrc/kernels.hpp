// kernels.hpp -- host-side launchers of the solver's HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace helm {

enum Prec { P64 = 0, P32 = 1, PBF = 2 };

// Up to MAXPTR device pointers passed by value as a kernel argument.
constexpr int MAXPTR = 32;
struct PtrList {
  const void* p[MAXPTR];
};

[[noreturn]] void fatal_combo(const char* where);

// Device allocation for every buffer of the library. With HELM_SENTINEL=1 in
// the environment (read at each call) the new memory is filled with 0xFF
// bytes, a NaN in FP64, FP32 and BF16, so that a kernel reading memory no
// kernel has written shows up as a non-finite result (write-coverage check).
hipError_t dmalloc_raw(void** p, size_t bytes);
template <class T> inline hipError_t dmalloc(T** p, size_t bytes) {
  return dmalloc_raw(reinterpret_cast<void**>(p), bytes);
}

// ---- k_level.hip ------------------------------------------------------------
// Tile shape of the 3D finest-level marching kernel (rows per lane 1/2/4,
// planes per z-chunk); results do not depend on it.
struct FineTile {
  int ry, zc;
};
void set_fine_tile(FineTile t);
// Fused 3D finest-level residual f - M u and full-weighting restriction into
// the coarse field rc (bitwise equal to the two separate kernels). Runs and
// returns true only for the LDS-blocked tiles and supported precisions.
bool can_resid_restrict(Prec pf, Prec pc, Prec pt, const Geo& gf);
bool launch_resid_restrict(Prec pf, Prec pc, Prec pt, const Geo& gf, const Geo& gc, const void* u, const void* f,
                           void* rc, const void* dg, const double ih[3], hipStream_t s);
// First post-smoothing sweep of the 3D finest level with the coarse-grid
// correction fused in: out = JAC(u + P ec) (bitwise the prolongation followed
// by the sweep). Runs and returns true only for the LDS-blocked tiles.
bool can_prolong_sweep(Prec pc, Prec pf, Prec pt, const Geo& gf);
bool launch_prolong_sweep(Prec pc, Prec pf, Prec pt, const Geo& gf, const Geo& gc, const void* ec, const void* u,
                          const void* f, void* out, const void* dg, const void* dw, const double ih[3],
                          hipStream_t s);
// The first two damped-Jacobi sweeps of the 3D finest level in one pass:
// out = JAC(w D^-1 f), bitwise the zero-guess sweep followed by a sweep.
// Available (can_sweep01) for the LDS-blocked tiles and FP32 / FP64 fields.
bool can_sweep01(Prec pf, Prec pt, const Geo& g);
// The two pre-sweeps from a zero guess, the residual and the restriction in
// one pass on the finest 3D level (k_pre_rr): u2 (the second sweep's result)
// into u2, the restricted residual into rc; bitwise the sweep01 +
// resid_restrict pair. Available where both of those are.
bool can_pre_rr(Prec pf, Prec pc, Prec pt, const Geo& gf);
bool launch_pre_rr(Prec pf, Prec pc, Prec pt, const Geo& gf, const Geo& gc, const void* f, void* u2, void* rc,
                   const void* dg, const void* dw, const double ih[3], hipStream_t s);
void launch_sweep01(Prec pf, Prec pt, const Geo& g, const void* f, void* out, const void* dg, const void* dw,
                    const double ih[3], hipStream_t s);
FineTile get_fine_tile();
// mode: 0 apply (out = A u), 1 residual (out = f - A u),
//       2 Jacobi (out = u + dw (f - A u)), 3 zero-guess Jacobi (out = dw f).
void launch_fine(int mode, Prec pu, Prec pf, Prec po, Prec pt, int dim, const Geo& g, const void* u, const void* f,
                 void* out, const void* diag, const void* dw, const double ih[3], hipStream_t s);
void launch_gal(int mode, Prec ps, Prec pt, int dim, const Geo& g, const void* u, const void* f, void* out,
                const void* st, const void* dw, hipStream_t s);
void launch_restrict(Prec pi, Prec po, Prec pt, int dim, const Geo& gf, const Geo& gc, const void* rf, void* rc,
                     hipStream_t s);
void launch_prolong_add(Prec pc, Prec pf, Prec pt, int dim, const Geo& gf, const Geo& gc, const void* ec, void* uf,
                        hipStream_t s);
void launch_convert(Prec pi, Prec po, int64_t nvals, const void* a, void* b, hipStream_t s);
// K-cycle: z1 <- y1 z1 + y2 z2 per column (Y: [2][P] complex), fields of N x P.
void launch_kc_combine(Prec pf, int64_t N, int P, const c128* Y, void* z1, const void* z2, hipStream_t s);
void launch_to_internal(Prec po, int64_t N, int nrhs, int P, const void* src, void* dst, hipStream_t s);
void launch_to_abi(Prec pi, int64_t N, int nrhs, int P, const void* src, void* dst, hipStream_t s);

// ---- k_resid.hip ------------------------------------------------------------
// Final FP64 residual check on the ABI layout: scratch[0..nrhs) receives
// relres_s = ||q_s - H u_s|| / ||q_s|| (0 for q_s = 0); scratch must hold
// resid_scratch_doubles(nrhs, N) doubles (the rest holds partial sums).
constexpr int RESID_MAX_COLS = 256;
constexpr int RESID_MAX_CHUNKS = 256;
int resid_chunks(int64_t N);
size_t resid_scratch_doubles(int nrhs, int64_t N);
void launch_resid_norms(const Geo& g, int nrhs, const double ih[3], const c128* dH, const void* Q, const void* U,
                        double* scratch, hipStream_t s);
// Device address, on the current device, of the library's static
// partial-sum array for launch_resid_norms (sized for RESID_MAX_COLS
// columns); looked up once per device.
hipError_t resid_static_scratch(double** out);

// ---- k_sens.hip -------------------------------------------------------------
// Sensitivity products (eq:fwisens) and 16-bit fields, ABI layout [nrhs][N].
void launch_sens_coef(int64_t N, const double* gamma, double omega, c128* dS, hipStream_t s);
void launch_jvp_rhs(int64_t N, int nrhs, const c128* dS, const void* U, const void* U16, const double* sc,
                    const double* dm, c128* out, hipStream_t s);
void launch_jtvp_accum(int64_t N, int nrhs, const c128* dS, const void* U, const void* U16, const double* sc,
                       const c128* Y, double* g, hipStream_t s);
void launch_conj(int64_t n, c128* x, hipStream_t s);
void launch_pack16(int64_t N, int nrhs, const c128* U, double* sc, void* H, hipStream_t s);
void launch_unpack16(int64_t N, int nrhs, const void* H, const double* sc, c128* U, hipStream_t s);

// ---- k_setup.hip ------------------------------------------------------------
// Fine-level diagonals from (m, gamma): dH, dM (shifted) and dw = wjac / dM.
void launch_fine_coef(int dim, int64_t N, const double* m, const double* gamma, double omega, double beta,
                      double wjac, const double ih[3], c128* dH, c128* dM, c128* dw, hipStream_t s);
// Galerkin stencil of the level below the fine one (from the 5/7-point M).
void launch_galerkin_from_fine(int dim, const Geo& gf, const Geo& gc, const c128* dM, const double ih[3], c128* stc,
                               hipStream_t s);
// Galerkin stencil from a 9/27-point level.
void launch_galerkin_from_gal(int dim, const Geo& gf, const Geo& gc, const c128* stf, c128* stc, hipStream_t s);
// dw[i] = wjac / st[i][centre].
void launch_gal_dw(int dim, int64_t N, const c128* st, double wjac, c128* dw, hipStream_t s);
// Dense row-major matrix of a stencil operator (n x n, n = npts).
void launch_assemble_dense(int dim, const Geo& g, const c128* st, c128* A, hipStream_t s);
// FP64 complex -> FP32 complex, elementwise (any length).
void launch_narrow(int64_t n, const c128* a, c64* b, hipStream_t s);
// In-place Gauss-Jordan inverse of a dense n x n matrix with block size nb,
// without pivoting (the shifted operators have a positive definite
// Hermitian part after multiplication by -i, so every pivot block is
// nonsingular). Workspace: n*nb*2 + nb*nb complex. Returns 0 or an error.
int gauss_jordan_inverse(int64_t n, c128* A, int nb, c128* work, hipStream_t s);
// C = alpha A B + beta C, row-major, complex (T = double or float storage
// c128 / c64). lda/ldb/ldc in elements.
void launch_gemm(Prec p, int64_t M, int64_t N, int64_t K, c128 alpha, const void* A, int64_t lda, const void* B,
                 int64_t ldb, c128 beta, void* C, int64_t ldc, hipStream_t s);

// ---- k_krylov.hip -----------------------------------------------------------
// Block Gram products per group of pb columns:
//   G[i][c][a] = sum_n conj(X_i[n][g*pb+a]) Y[n][c],  g = c / pb, c < P,
// for k <= MAXPTR matrices X_0..X_{k-1}, FP64 c128 [N][ld].
// `part` is scratch (>= gram_part_elems complex); G has k * P * pb entries.
// Storage p = P64 (c128) or P32 (c64); accumulation is FP64.
int64_t gram_part_elems(int P);
void launch_gram(Prec p, int64_t N, int ld, int P, int pb, int k, const PtrList& X, const void* Y, c128* part,
                 c128* G, hipStream_t s);
// Y[n][c] (+/-)= sum_i sum_a X_i[n][g*pb+a] C_i[c][a]  (C layout as G).
//   mode 0: Y -= ..., mode 1: Y = ... (overwrite), mode 2: Y += ...
// X may be c128 or c64 (px), Y c128 or c64 (py); arithmetic in FP64.
void launch_block_update(int mode, Prec px, Prec py, int64_t N, int ld, int P, int pb, int k, const PtrList& X,
                         const c128* C, void* Y, hipStream_t s);
// Per group g < ng: Cholesky G_g = R^H R (pb x pb, G layout [c][a] of one X),
// R and Rinv written [g][pb][pb] row-major (row a, col b). flag[g] = 1 on
// breakdown (pivot <= tol * max diagonal).
void launch_cholqr_small(int ng, int pb, const c128* G, c128* R, c128* Rinv, int* flag, double tol, double rtol,
                         hipStream_t s);
void launch_rmul_small(int ng, int pb, const c128* R2, c128* R, hipStream_t s);
// Block FGMRES least squares per group: Hbar_g is ((j+2)pb x (j+1)pb),
// column-major with leading dimension ldh, stored at Hb + g*hstride; S_g the
// pb x pb first block (row-major). Writes Y_g ((j+1)pb x pb, column-major
// ld (j+1)pb... stored at Y + g*ystride) and est[g*pb+b] = residual norm of
// column b. scratch: per group (j+2)pb*((j+1)pb + pb) complex.
void launch_block_ls(int ng, int pb, int j, const c128* Hb, int ldh, int64_t hstride, const c128* S, c128* Y,
                     int64_t ystride, double* est, c128* scratch, const int* active, hipStream_t s);
// Column norms^2 of a block (P columns of [N][ld]) -> out[P] (double).
// G: scratch of P complex.
void launch_colnorm2(Prec p, int64_t N, int ld, int P, const void* X, c128* part, c128* G, double* out,
                     hipStream_t s);
// out[c] = Re G[c], c < P.
void launch_diag_real(int P, const c128* G, double* out, hipStream_t s);
// Columns with active[g]==0 are zeroed in Y (inactive groups of the block).
void launch_mask_cols(int64_t N, int ld, int P, int pb, const int* active, c128* Y, hipStream_t s);
// Scale columns: Y[n][c] = s[c] * X[n][c] (in place allowed).
void launch_scale_cols(Prec p, int64_t N, int ld, int P, const double* sc, const void* X, void* Y, hipStream_t s);
// Block size 1: Y -= sum_i X_i C_i (per column) and nrm2[c] = ||Y_c||^2 after
// the update (part: gram_part_elems scratch; G: P complex scratch).
void launch_update_norm(Prec p, int64_t N, int ld, int P, int k, const PtrList& X, const c128* C, void* Y,
                        c128* part, c128* G, double* nrm2, hipStream_t s, const double* osc = nullptr);
void launch_cg_lazy_init(int P, const double* b2, double* nu, hipStream_t s);
void launch_cg_lazy_coef(int P, int j, c128* Gc, const double* nu, double* osc, hipStream_t s);
void launch_cg_lazy_hcol(int P, int j, int k, const c128* Gc, const double* hn2, double* nu, c128* H,
                         hipStream_t s);
// R = ||w||, Rinv = 1/||w|| per column from n2; flag where n2 <= tol*ref2.
void launch_norm_to_r(int P, const double* n2, const double* ref2, double tol, c128* R, c128* Rinv, int* flag,
                      hipStream_t s);
// Block size 1 with an unnormalised Krylov basis (see k_krylov.hip).
void launch_lazy_coef(int P, int j, const c128* Graw, const double* nu, c128* C, c128* Hb, int ldh, int64_t hstride,
                      int accumulate, hipStream_t s);
void launch_lazy_next(int P, int j, const double* n2, const double* ref2, double tol, double* nu, c128* Hb, int ldh,
                      int64_t hstride, int* flag, hipStream_t s);
void launch_lazy_start(int P, const double* r2, double* nu, c128* S, int* flag, hipStream_t s);
void launch_lazy_y(int P, int k, const double* nu, c128* Y, hipStream_t s);
// ---- k_bicg.hip -------------------------------------------------------------
// Block BiCGSTAB per group of pb columns (matrices in the Gram layout):
// X_g = sgn A_g^-1 B_g (zero for an inactive group or, flag[g] = 1, a
// singular A_g); omega_g = trace(T^H S) / trace(T^H T); coefficient lists
// (kind 0..3, see k_bicg.hip) for launch_block_update.
void launch_bicg_solve(int ng, int pb, double sgn, const c128* A, const c128* B, c128* X, const int* act, int* flag,
                       hipStream_t s);
void launch_bicg_omega(int ng, int pb, const c128* Gts, const double* tn2, const int* act, c128* om, hipStream_t s);
void launch_bicg_coefs(int kind, int P, int pb, const c128* M, const c128* om, c128* C, hipStream_t s);

// Fixed-step per-column GMRES helpers for the coarsest grid.
void launch_cg_hcol(int P, int j, int k, const c128* Gc, const double* hn2, c128* H, double* sc, hipStream_t s);
void launch_inv_sqrt(int P, const double* b2, double* sc, hipStream_t s);
// Per-column least squares of the fixed-step GMRES: H ((k+1) x k per column)
// is rotated in place; G is scratch of (k+1) * P complex.
void launch_cg_ls(int P, int k, c128* H, const double* b2, c128* G, c128* Y, hipStream_t s);

// ---------------------------------------------------------------------------
// Persistent cycle: the launches of one multigrid cycle recorded as phases
// that one cooperative kernel runs in order, a grid-wide barrier after each.
// Every phase runs the per-item code of the stand-alone kernel it replaces
// (fine_item, gal_item, restrict_item, prolong_item, gemm_tile).
// ---------------------------------------------------------------------------
enum PhaseOp : int { PH_FINE = 0, PH_GAL = 1, PH_RESTRICT = 2, PH_PROLONG = 3, PH_ZERO = 4, PH_GEMM = 5 };
struct Phase {
  int op;            // PhaseOp
  int mode;          // operator mode (FINE, GAL): 0 apply, 1 residual, 2 Jacobi, 3 Jacobi from zero
  int pa, pb;        // Prec: field (FINE, GAL); in / out (RESTRICT); coarse / fine (PROLONG); GEMM storage
  Geo g, gc;         // level (fine side of a transfer), coarse side of a transfer
  const void* u;     // FINE/GAL: u; RESTRICT: fine residual; PROLONG: coarse correction; GEMM: B
  const void* f;     // FINE/GAL: right-hand side
  void* out;         // output (ZERO: the 16-byte units to clear; PROLONG: the fine field, updated)
  const void* c0;    // FINE: diagonal; GAL: stencil; GEMM: A (the coarsest inverse)
  const void* c1;    // FINE/GAL: w / diagonal
  double ih[3];      // FINE: 1/h^2 per axis
  int64_t n;         // ZERO: 16-byte units; GEMM: order of A
};
// Grid size of the persistent kernel for (dim, mixed): the workgroups that
// are co-resident on the device (0 if the device cannot launch it).
int persist_grid(int dim, bool mixed);
// Runs the nph phases at ph (device memory) with a cooperative launch of
// `grid` workgroups; returns the launch status.
hipError_t launch_cycle_persist(int dim, bool mixed, const Phase* ph, int nph, int grid, hipStream_t s);

}  // namespace helm
