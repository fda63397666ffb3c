/*
 * helm.h -- C ABI of the MI355X block shifted-Laplacian Helmholtz solver.
 *
 * Problem (Treister & Haber, "Full waveform inversion guided by travel time
 * tomography", eq:helm and eq:LinearSystem): for many right-hand sides q_s
 * solve H u_s = q_s with
 *     H = -Lap_h - omega^2 diag(m (1 - i gamma)),
 * the second-order 5-point (2D) / 7-point (3D) finite-difference Laplacian on
 * a vertex-centred grid with homogeneous Dirichlet values outside. gamma is
 * dimensionless (the paper's gamma/omega) and carries the absorbing layer;
 * the paper's sign convention differs by negating q.
 *
 * Method (section "Solving the Helmholtz equation for multiple right hand
 * sides" and section 5.3): block FGMRES(m) right-preconditioned by a
 * multigrid cycle for the shifted operator M = H with gamma -> gamma + shift
 * (the paper adds a positive constant to gamma; 0.2 in its experiments).
 * The cycle uses damped Jacobi relaxation (weight 0.8, 2 pre + 2 post),
 * full-weighting restriction R = 2^-d P^T, d-linear prolongation P, Galerkin
 * coarse operators R M P (the two-grid cycle algorithm, recursively) and an
 * LU-based solve of the coarsest grid for the whole block.
 *
 * Conventions for every entry point:
 *  - Every call returns helm_status; nothing throws across the ABI. On error
 *    helm_last_error() returns a thread-local message.
 *  - Complex numbers are interleaved (re, im) doubles.
 *  - Blocks of right-hand sides / solutions are DEVICE arrays of complex128
 *    laid out [nrhs][N]: each right-hand side contiguous, grid axis 0 fastest
 *    (N = prod(n[a]-1)). The library converts to its own internal layout.
 *  - Setup inputs (m, gamma) are HOST FP64 arrays of N entries, copied in.
 *  - `stream` is a hipStream_t (NULL = default stream). All device work of a
 *    call is ordered on that stream; calls that return host values
 *    synchronise it.
 *  - The caller owns Q, U and any workspace; the handle owns the hierarchy.
 *  - One handle must not be used by two threads at once.
 *  - Debugging aid: with the environment variable HELM_SENTINEL=1 (read at
 *    every allocation), each device buffer the library allocates starts
 *    filled with 0xFF bytes (NaN in FP64, FP32 and BF16) instead of whatever
 *    the allocator returns, so a read of memory no kernel has written shows
 *    as a non-finite result. Results are otherwise unchanged.
 *  - Check aid: with HELM_NET_CONCAT=1 (read at every network forward pass of
 *    helm_net_forward and of the learned coarsest solve) the network's
 *    inference pass takes the form its training pass uses, with the decoder
 *    inputs copied into concatenated buffers; the outputs are bitwise equal
 *    to the default form, which reads those inputs in place.
 */
#ifndef HELM_H
#define HELM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HELM_MAX_LEVELS 8

typedef struct helm_ctx* helm_handle;

typedef enum {
  HELM_OK = 0,
  HELM_ERR_INVALID_ARG = 1,   /* bad shape, level count, pointer or option  */
  HELM_ERR_OOM = 2,           /* device allocation failed                   */
  HELM_ERR_DEVICE = 3,        /* a HIP runtime call or kernel launch failed */
  HELM_ERR_NOT_CONVERGED = 4, /* U holds the last iterate, info is filled   */
  HELM_ERR_BREAKDOWN = 5,     /* a block BiCGSTAB breakdown (e.g. dependent sources in one block), or a divergence
                                 that could not be handled (U holds the last good iterate) */
  HELM_ERR_NONFINITE = 6,     /* NaN/Inf in m, gamma or Q                    */
  HELM_ERR_UNSUPPORTED = 7    /* valid request the library does not support */
} helm_status;

enum { HELM_FP64 = 0, HELM_MIXED = 1 };
/* Coarsest-grid solve: exact (dense inverse of the Galerkin operator, FP64
 * Gauss-Jordan at setup, applied as one matrix product for the block),
 * learned network, none (the coarsest level is only relaxed), or
 * coarse_iters steps of GMRES from zero per column (an inexact iterative
 * coarsest solve, which the paper discusses in section 5.3 for coarse grids
 * too large to factor). */
enum { HELM_COARSE_LU = 0, HELM_COARSE_LEARNED = 1, HELM_COARSE_NONE = 2, HELM_COARSE_GMRES = 3 };
/* Cycle shape below the finest level: V (one recursive call), W (two; the
 * two-grid cycle text), or K (the paper's K-FGMRES of section 5.3: every
 * coarse level but the coarsest is solved by two flexible GMRES steps from
 * zero per column, each preconditioned by that level's cycle; a nonlinear
 * preconditioner, for FGMRES). */
enum { HELM_CYCLE_V = 0, HELM_CYCLE_W = 1, HELM_CYCLE_K = 2 };

typedef struct {
  int32_t dim;                 /* 2 or 3 */
  int32_t n[3];                /* cells per axis, axis 0 fastest; unknowns n-1;
                                  n[a] % 2^(levels-1) == 0; n[2] ignored in 2D */
  double h[3];                 /* spacing per axis (> 0) */
  const double* m;             /* HOST [N] squared slowness (> 0) */
  const double* gamma;         /* HOST [N] dimensionless attenuation (>= 0) */
  double omega;                /* angular frequency (> 0) */
  double shift;                /* beta >= 0 added to gamma in the preconditioner */
  int32_t levels;              /* 2..HELM_MAX_LEVELS; coarsest must have >= 1 unknown/axis */
  int32_t nu_pre[HELM_MAX_LEVELS];      /* Jacobi sweeps before the coarse correction */
  int32_t nu_post[HELM_MAX_LEVELS];     /* and after it */
  double jacobi_weight[HELM_MAX_LEVELS];/* damping per level (paper: 0.8) */
  int32_t precision;           /* HELM_FP64 or HELM_MIXED (FP32 cycle, BF16 fields at
                                  levels >= 2, FP64 outer Krylov) */
  int32_t coarse;              /* HELM_COARSE_* */
  int32_t cycle;               /* HELM_CYCLE_* */
  int32_t coarse_iters;        /* HELM_COARSE_GMRES: GMRES steps from zero (1..32);
                                  HELM_COARSE_LEARNED: GMRES steps started from the
                                  network's correction (0..32, 0 = network alone);
                                  larger values return HELM_ERR_INVALID_ARG */
  const void* net;             /* HOST weights blob for HELM_COARSE_LEARNED (or NULL) */
  size_t net_bytes;
  int32_t coarse_restarts;     /* GMRES and learned coarsest solves: restarted GMRES,
                                  this many cycles of coarse_iters steps, each on the
                                  current coarsest residual (0..16; 0 and 1: one cycle).
                                  The learned fallback stays max(k, 20) steps from zero. */
} helm_setup_desc;

/* Fill `d` with the paper's defaults: shift 0.2, 2+2 sweeps at 0.8, V-cycle,
 * FP64, LU coarsest (20 GMRES steps, one cycle, if HELM_COARSE_GMRES is
 * chosen), 3 levels. Geometry, m, gamma and omega are left zero. */
void helm_setup_desc_default(helm_setup_desc* d);

typedef struct {
  int32_t restart;     /* m of FGMRES(m), 1..31 (paper: 5) */
  int32_t max_cycles;  /* cap on preconditioner applications (Arnoldi steps) */
  int32_t block_size;  /* RHS per Krylov block; must divide nrhs, <= 64 (0 = nrhs). FGMRES
                          orthonormalises each new block by CholQR and deflates: a column
                          whose part independent of the block's earlier columns is at most
                          1e-6 of its norm is dropped from the basis (a second CholQR pass
                          follows such a drop, or a near-dependence), so duplicate or
                          dependent sources in one block are solved */
  int32_t warm_start;  /* 1: U holds an initial guess */
  int32_t reorth;      /* 0: one block Gram-Schmidt pass; 1: always two; 2: a second
                          pass only where the norm fell below half (block size 1) */
  int32_t graph;       /* execution form of the cycle. 0: eager launches. 1: a HIP graph
                          captured on first use per (block width, buffers) and replayed
                          afterwards; results are bitwise those of the eager launches.
                          2: one cooperative launch of a persistent kernel per cycle that
                          runs the cycle's steps with grid-wide barriers between them
                          (V-cycle with the LU coarsest solver only, else
                          HELM_ERR_INVALID_ARG; not in helm_solve_batch); in 2D its
                          results are bitwise those of the eager launches, in 3D they
                          differ by rounding (the eager path uses the tiled and fused
                          kernels there). 1 and 2 are ignored while kernel timing
                          (helm_profile_enable) or pair capture is on. */
  double learned_rate; /* learned coarsest correction only: the calibrated per-cycle
                          residual reduction factor rho of the plain cycle (0 < rho < 1,
                          e.g. tol^(1/cycles) of a solve with the LU or GMRES coarsest
                          solver); 0 turns the check off. At every restart the solve
                          measures its own factor, (max_s relres_s now / at the previous
                          restart)^(1 / cycles in between); when that is above sqrt(rho),
                          i.e. the solve would need more than twice the calibrated
                          cycles, the coarsest solves switch to the GMRES fallback for
                          the rest of the solve (info.rate_switch). */
  int32_t method;      /* HELM_METHOD_FGMRES (0): block FGMRES(restart). HELM_METHOD_BICGSTAB (1):
                          block BiCGSTAB (the paper's W-BiCG with cycle = HELM_CYCLE_W; El
                          Guennouni, Jbilou and Sadok's block version), two cycles per
                          iteration, groups of block_size columns; restart and reorth are
                          ignored. BiCGSTAB is not flexible: its theory needs a linear cycle
                          (LU or relaxation-only coarsest solve); with the GMRES or learned
                          coarsest solve it runs with a fixed but nonlinear cycle, and the
                          FP64 true residual, checked whenever the recursive one meets tol
                          (then restarting from the current iterate if needed), keeps the
                          result honest either way. */
  int32_t op;          /* the system solved: HELM_OP_H (0) H U = Q; HELM_OP_HT (1) the
                          transposed system H^T U = Q, the same system because H is complex
                          symmetric (a symmetric stencil plus a diagonal) and so is every
                          Galerkin level (R = 2^-d P^T), so the hierarchy serves both, as the
                          paper notes for the transposed solves of its sensitivities;
                          HELM_OP_HH (2) the adjoint H^H U = Q, solved as H conj(U) = conj(Q)
                          (the reported relres is that of the adjoint system) */
} helm_solve_opts;

enum { HELM_METHOD_FGMRES = 0, HELM_METHOD_BICGSTAB = 1 };
enum { HELM_OP_H = 0, HELM_OP_HT = 1, HELM_OP_HH = 2 };

typedef struct {
  int32_t cycles;       /* preconditioner applications (the paper's #Cyc): Arnoldi steps of
                           FGMRES, two per BiCGSTAB iteration */
  int32_t restarts;
  int32_t converged_all;
  int32_t fallback_used;/* coarsest solves where the learned correction was not finite
                           or beyond 1e4 in its normalised units, and max(coarse_iters,
                           20) GMRES steps from zero replaced it */
  double t_solve_ms;    /* device time of the solve (hip events) */
  double* relres;       /* HOST [nrhs] or NULL: final FP64 ||q_s - H u_s|| / ||q_s|| */
  int32_t* converged;   /* HOST [nrhs] or NULL */
  int32_t rate_switch;  /* cycles done when the learned_rate check switched to the
                           fallback, or -1 */
} helm_solve_info;

/* Build the hierarchy: fine coefficients, Galerkin operators per level
 * (two-grid cycle text: A_c = P^T A P), and the coarsest solve (LU of the
 * coarsest grid for a block of RHS). Synchronises `stream`. */
helm_status helm_setup(const helm_setup_desc* desc, void* stream, helm_handle* out);
void helm_destroy(helm_handle h);

/* Bytes of device workspace helm_solve_block needs for `nrhs`, `restart`. */
helm_status helm_workspace_size(helm_handle h, int32_t nrhs, int32_t restart, size_t* bytes);

/* Solve H U = Q (block FGMRES, section 5.3) until every column satisfies
 * ||q_s - H u_s|| / ||q_s|| <= tol in FP64 (a zero column is converged at 0).
 * Q, U: DEVICE complex128 [nrhs][N]. workspace: DEVICE, >= helm_workspace_size
 * bytes, or NULL to let the handle allocate and cache it. info: HOST, may be
 * NULL. Returns HELM_ERR_NOT_CONVERGED (U = last iterate) if max_cycles is hit. */
helm_status helm_solve_block(helm_handle h, int32_t nrhs, const void* Q, void* U, double tol,
                             const helm_solve_opts* opts, void* workspace, size_t ws_bytes,
                             helm_solve_info* info, void* stream);

/* Set up k hierarchies, one per descriptor (for example one model at the
 * frequencies of a frequency-continuation sweep, the paper's frequency
 * continuation algorithm, each frequency with its own hierarchy), as k
 * calls of helm_setup on `stream`. out: HOST [k]. On an error no handle is
 * left: the ones already built are destroyed, out[] is NULL and the
 * message names the instance. */
helm_status helm_setup_batch(int32_t k, const helm_setup_desc* descs, void* stream, helm_handle* out);

/* Solve k independent instances concurrently (uneven sizes welcome): instance
 * i is helm_solve_block(hs[i], nrhs[i], Q[i], U[i], tol, opts) on a stream
 * owned by hs[i] (created on first use, default priority), driven by a pool of
 * min(k, max_threads) host threads (max_threads <= 0: 16). The handles must be
 * distinct. Work queued on `stream` before the call is visible to every
 * instance, and `stream` waits for all of them. Q[i], U[i]: DEVICE complex128
 * [nrhs[i]][N_i]; infos: HOST [k] or NULL (each entry as for
 * helm_solve_block); status: HOST [k] or NULL, per-instance results. Returns
 * the first non-OK instance status (its message prefixed with the index), or
 * HELM_OK. Results are bitwise those of solving the instances one by one. */
helm_status helm_solve_batch(int32_t k, const helm_handle* hs, const int32_t* nrhs, const void* const* Q,
                             void* const* U, double tol, const helm_solve_opts* opts,
                             helm_solve_info* infos, int32_t* status, int32_t max_threads,
                             void* stream);

/* The stopping rule's quantity (section 5.3: a solve ends when the initial
 * residual is reduced by the tolerance; here per column, from U = 0), in
 * FP64: relres[s] = ||q_s - H u_s||_2 / ||q_s||_2 with H of eq:helm /
 * eq:LinearSystem (0 for a zero q_s; NaN where Q or U holds a NaN).
 * Q, U: DEVICE complex128 [nrhs][N], 1 <= nrhs <= 256, read once in place;
 * relres: HOST [nrhs]. The handle allocates a partial-sum buffer of about
 * 1 MB on the first call and keeps it. Synchronises `stream`. */
helm_status helm_residual(helm_handle h, int32_t nrhs, const void* Q, const void* U,
                          double* relres, void* stream);

/* helm_residual for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and bitwise the same relres, but its partial sums live in
 * a static device array of the library (about 1 MB per device, held until
 * the process ends) instead of the handle's buffer. It calls no hipMalloc,
 * hipFree or other allocating routine. nrhs beyond 256 (the array's size)
 * returns HELM_ERR_INVALID_ARG. Every call on one device shares that
 * device's array: calls that overlap on one device (other streams, other
 * threads) race and must be serialised by the caller. Synchronises
 * `stream`. */
helm_status helm_residual_noalloc(helm_handle h, int32_t nrhs, const void* Q, const void* U,
                                  double* relres, void* stream);

/* ---- Sensitivities of full waveform inversion (eq:fwisens) -----------------
 * With H u = q and dH/dm = -omega^2 diag(1 - i gamma) (m the squared
 * slowness, real), the Jacobian of the field in the model is
 *     J dm  = omega^2 H^-1 ((1 - i gamma) u . dm)        (one solve per source)
 *     J^H w = omega^2 conj((1 - i gamma) u) . H^-H w     (one adjoint solve each)
 * Fields u_s are given either in complex128 (U) or in the paper's 16-bit
 * storage (U16 + scales, see helm_fields_pack16); exactly one of U and U16
 * is non-NULL. The solves use helm_solve_block with the given tol and opts
 * (opts.op is set by the call); info as there. */

/* 16-bit storage of fields (the paper stores fields in a 16-bit floating
 * point format, 32 bits per complex unknown and source): per source,
 * scales[s] = the largest |re| or |im| of u_s (1 for a zero source), and
 * U16[s][i] = (half(re / scales[s]), half(im / scales[s])), each value
 * formed in FP64, rounded to FP32 and then to IEEE half (nearest even).
 * U: DEVICE complex128 [nrhs][N]; U16: DEVICE 2 x FP16 [nrhs][N] (4 bytes per
 * entry, re first); scales: DEVICE double [nrhs]. */
helm_status helm_fields_pack16(helm_handle h, int32_t nrhs, const void* U, void* U16, double* scales,
                               void* stream);
/* U[s][i] = scales[s] * (re + i im) of U16[s][i], in FP64. */
helm_status helm_fields_unpack16(helm_handle h, int32_t nrhs, const void* U16, const double* scales, void* U,
                                 void* stream);
/* JV[s] = J_s dm for every source: dm DEVICE double [N] (a real model
 * perturbation of m), JV DEVICE complex128 [nrhs][N] (also the solve's
 * right-hand side buffer). */
helm_status helm_jvp(helm_handle h, int32_t nrhs, const void* U, const void* U16, const double* scales,
                     const double* dm, void* JV, double tol, const helm_solve_opts* opts, helm_solve_info* info,
                     void* stream);
/* g = Re sum_s J_s^H w_s (the gradient of a real misfit with residuals w_s):
 * W DEVICE complex128 [nrhs][N], g DEVICE double [N]. The adjoint solutions
 * live in a buffer the handle allocates on first use and keeps. */
helm_status helm_jtvp(helm_handle h, int32_t nrhs, const void* U, const void* U16, const double* scales,
                      const void* W, double* g, double tol, const helm_solve_opts* opts, helm_solve_info* info,
                      void* stream);

/* Y = H X (op 0) or Y = M X (op 1, shifted), in FP64 (eq:LinearSystem).
 * X, Y: DEVICE complex128 [nrhs][N]. */
helm_status helm_apply(helm_handle h, int32_t op, int32_t nrhs, const void* X, void* Y,
                       void* stream);

/* Z = one multigrid cycle applied to R (the preconditioner, in the handle's
 * precision). R, Z: DEVICE complex128 [nrhs][N]. */
helm_status helm_precond(helm_handle h, int32_t nrhs, const void* R, void* Z, void* stream);

/* Unknowns per axis of level l (0 = finest). */
helm_status helm_level_dims(helm_handle h, int32_t level, int32_t nu[3]);

/* Copy the operator of level l >= 1 to HOST `st` as FP64 complex
 * [N_l][3^dim] (entry (ox+1) + 3(oy+1) [+ 9(oz+1)] couples node i to node
 * i + offset), converted from the stored precision. */
helm_status helm_level_stencil(helm_handle h, int32_t level, double* st);

/* E = coarsest-grid solve applied to R (as used inside the cycle).
 * R, E: DEVICE complex128 [nrhs][N_coarsest]. */
helm_status helm_coarse_solve(helm_handle h, int32_t nrhs, const void* R, void* E, void* stream);

/* Tile shape (rows per lane, planes per z-chunk) of the 3D finest-level
 * stencil kernels for blocks of nrhs columns. helm_fine_tile runs the
 * autotuner if this width has not been tuned (timing each candidate on the
 * handle's buffers; cached in the JSON-lines file named by HELM_TUNE_CACHE;
 * HELM_AUTOTUNE=0 keeps the default) and returns the choice;
 * helm_set_fine_tile forces one (ry in {1,2,4}: rows per lane of the
 * register-blocked kernel; ry = 16 or 8: the LDS-blocked kernel on 16 x 16 or
 * 16 x 8 tiles, used where the block width is a multiple of 128 B of
 * right-hand sides;
 * zc >= 1). Results are bitwise identical for every tile. With the
 * LDS-blocked tiles the finest-level residual runs fused with the
 * restriction, and the prolongation with the first post-smoothing sweep;
 * the environment variable HELM_FUSE=0 (read once per process) runs them as
 * separate kernels instead, again with bitwise identical results. */
helm_status helm_fine_tile(helm_handle h, int32_t nrhs, int32_t tile[2]);
helm_status helm_set_fine_tile(helm_handle h, int32_t nrhs, const int32_t tile[2]);

/* Per-class kernel timing with HIP events recorded on the solve's stream
 * around every launch of the class (for roofline accounting). */
enum {
  HELM_K_FINE_SWEEP = 0, /* damped-Jacobi sweeps from a nonzero guess, finest level */
  HELM_K_FINE_RESID,     /* residual of the cycle on the finest level */
  HELM_K_OUTER_APPLY,    /* W = H Z and R = Q - H X of the outer Krylov (FP64) */
  HELM_K_TRANSFER,       /* restriction and prolongation, all levels */
  HELM_K_COARSE_SWEEP,   /* relaxation / residual on Galerkin levels */
  HELM_K_COARSEST,       /* the whole coarsest-grid solve */
  HELM_K_GRAM,           /* block Gram products and column norms */
  HELM_K_UPDATE,         /* block updates W -= V H, V = W R^-1, X += Z Y */
  HELM_K_FINE_SWEEP0,    /* the first (zero initial guess) sweep on the finest level */
  HELM_K_FINE_PROSWEEP,  /* the first post-smoothing sweep with the prolongation fused in */
  HELM_K_FINE_SWEEP01,   /* the zero-guess sweep and the next sweep fused in one pass (3D,
                            LDS-blocked tiles) */
  HELM_K_FINE_PRE_RR,    /* the two pre-sweeps from a zero guess, the residual and the
                            restriction fused in one pass (3D, exactly two pre-sweeps) */
  HELM_K_NCLASS
};
typedef struct {
  int32_t launches;
  double total_ms;
} helm_kernel_stat;
/* enable != 0 starts timing (counters reset); 0 stops it. */
helm_status helm_profile_enable(helm_handle h, int32_t enable);
/* Fill stats[HELM_K_NCLASS]; synchronises the device. */
helm_status helm_profile_read(helm_handle h, helm_kernel_stat* stats);

const char* helm_status_string(helm_status s);
const char* helm_last_error(void);

/* ---- Learned coarsest-grid correction ------------------------------------
 * The paper names a cheaper stationary inexact solver of the coarsest grid as
 * future work (end of section 5.3 and the conclusions). This is one: a 3-level
 * 3D U-Net (channels 16/32/64, 3x3x3 convolutions + ReLU, 2x average pooling,
 * nearest upsampling, skip connections by concatenation, a linear 1x1 head)
 * on a D^3 volume that embeds the coarsest grid (D = its largest unknown count
 * per axis rounded up to a multiple of 4). Input channels per voxel: Re, Im of
 * r / rms(r) and Re, Im of H^2 times the diagonal of the coarsest Galerkin
 * operator; output e = H^2 rms(r) (out_0 + i out_1). BF16 activations and
 * weights, FP32 accumulation and master weights. Parameters are packed per
 * 3x3x3 layer as W[27][Cin][Cout] (tap (dx+1) + 3(dy+1) + 9(dz+1), x fastest)
 * then b[Cout], then the head W[16][2], b[2].
 * A network is used by helm_setup with coarse = HELM_COARSE_LEARNED and
 * net = a blob from helm_net_save (3D only). With coarse_iters = k > 0 the
 * network's correction is the initial guess of k GMRES steps on the coarsest
 * grid. An output that is not finite, or beyond 1e4 in the normalised units
 * e / (H^2 rms(r)), makes that coarsest solve fall back to max(k, 20) GMRES
 * steps from zero (counted in info.fallback_used); so does every coarsest
 * solve after the per-cycle rate check of helm_solve_opts.learned_rate fired. */
typedef struct helm_net_s* helm_net;
/* Number of FP32 parameters. */
int64_t helm_net_nparams(void);
/* A network on D^3 volumes (D % 4 == 0, 4..256) for batches of up to
 * max_batch samples, He-initialised from seed. Synchronises `stream`. */
helm_status helm_net_create(int32_t D, int32_t max_batch, uint64_t seed, void* stream, helm_net* out);
void helm_net_destroy(helm_net n);
/* HOST [helm_net_nparams()] FP32 parameters in the packing above. Setting
 * resets the optimiser state. */
helm_status helm_net_set_params(helm_net n, const float* params);
helm_status helm_net_get_params(helm_net n, float* params);
/* Training checkpoint (the Adam update of helm_net_train_step and
 * helm_net_train). state: HOST [3 * helm_net_nparams()] FP32 = the
 * parameters, then Adam's first moments, then its second moments; step: the
 * update count t of the bias correction. get_state copies them out;
 * set_state restores them (parameters and first moments finite, second
 * moments finite and >= 0, step >= 0, else an error and nothing changes), so
 * that training resumed from a checkpoint takes the same updates, bitwise, as
 * training that never stopped. */
helm_status helm_net_get_state(helm_net n, float* state, int64_t* step);
helm_status helm_net_set_state(helm_net n, const float* state, int64_t step);
/* Serialise: blob == NULL returns the size in *bytes; otherwise writes
 * "HNET", uint32 1, int64 nparams, float params[] into blob (HOST). */
helm_status helm_net_save(helm_net n, void* blob, size_t* bytes);
/* out = network(x). x: DEVICE FP32 [B][D^3][4], out: DEVICE FP32 [B][D^3][2],
 * 1 <= B <= max_batch. Synchronises `stream`. */
helm_status helm_net_forward(helm_net n, int32_t B, const float* x, float* out, void* stream);
/* loss = (1/B) sum_s ||out_s - t_s||^2 / ||t_s||^2 over voxels with mask != 0
 * (samples with t_s = 0 on the mask add 0) and grad = d loss / d params.
 * x, target as above, mask: DEVICE uint8 [D^3], grad: DEVICE FP32 [nparams],
 * loss: HOST. Synchronises `stream`. */
helm_status helm_net_loss_grad(helm_net n, int32_t B, const float* x, const float* target,
                               const uint8_t* mask, float* grad, double* loss, void* stream);
/* One training step on a caller-supplied minibatch (buffers as for
 * helm_net_loss_grad; no sampling and no phase rotation): the loss and its
 * gradient, then one Adam update (Kingma & Ba: beta 0.9, 0.999, eps 1e-8,
 * bias-corrected moments; step t counts every update since the parameters
 * were last set) of the FP32 master weights and their BF16 working copies.
 * loss: HOST, may be NULL. Synchronises `stream`. */
helm_status helm_net_train_step(helm_net n, int32_t B, const float* x, const float* target, const uint8_t* mask,
                               double lr, double* loss, void* stream);
/* Training pairs from a solver: until the next call, every coarsest solve of
 * `h` (3D; coarse must be LU or GMRES; its coarsest grid must fit D) stores
 * (input volume, exact-solve target) of each nonzero column into a pool of
 * max_pairs volumes held by n (reservoir sampling). max_pairs == 0 detaches;
 * max_pairs < 0 attaches to h and keeps n's existing pool (h's coarsest grid
 * must have the pool's dimensions), so that one pool holds the pairs of
 * several problems. */
helm_status helm_net_capture(helm_handle h, helm_net n, int32_t max_pairs);
int64_t helm_net_pairs(helm_net n);
/* Copy pool entry i (0 <= i < helm_net_pairs): x DEVICE FP32 [D^3][4] (the
 * network input as stored, BF16 widened) and target DEVICE FP32 [D^3][2]
 * (e / (H^2 rms(r)), 0 outside the grid). Synchronises `stream`. */
helm_status helm_net_pool_read(helm_net n, int64_t i, float* x, float* target, void* stream);
/* Adam (beta 0.9, 0.999, eps 1e-8) on minibatches of `batch` pool samples
 * drawn uniformly with `seed`; each sample's residual channels and target are
 * multiplied by one random unit phase (the exact coarsest solve commutes with
 * it, so the rotated pair is as valid as the stored one). hist: HOST [steps]
 * loss per step, or NULL. */
helm_status helm_net_train(helm_net n, int32_t steps, int32_t batch, double lr, uint64_t seed,
                           double* hist, void* stream);

#ifdef __cplusplus
}
#endif
#endif
