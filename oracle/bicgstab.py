"""Oracle of block BiCGSTAB with a stationary multigrid preconditioner (test
infrastructure only: only tests/, the smoke check and the benchmark's CPU
baseline use oracle/; the solver library never imports or calls it).

The paper's fastest configuration (section 5.3, table tab:MGperformance,
and the conclusions) is "W-BiCG": the block BiCGSTAB method of El
Guennouni, Jbilou and Sadok (ETNA 16, 2003) preconditioned by a multigrid
cycle, which must be stationary (a fixed linear map) because BiCGSTAB is
not flexible (end of section 5.3). The method, for a block of s right-hand
sides B and right preconditioning by M (the cycle), in plain FP64 numpy
around the oracle's pinned C primitives (the operator and the cycle):

  R = B - H X, shadow block Rt = R, P = R; then per iteration
    Phat = M P,  V = H Phat
    alpha  = (Rt^H V)^-1 (Rt^H R)                       (s x s)
    S = R - V alpha
    Shat = M S,  T = H Shat
    omega = trace(T^H S) / trace(T^H T)                 (scalar)
    X = X + Phat alpha + omega Shat
    R = S - omega T
    beta  = -(Rt^H V)^-1 (Rt^H T)                       (s x s)
    P = R + (P - omega V) beta
  until every column has ||r_c|| <= tol ||b_c||.

Each iteration applies the cycle twice; `cycles` counts those applications
(the paper's #Cyc counts preconditioning cycles). The small s x s systems
are solved by numpy.linalg.solve (LU with partial pivoting). The residual R
is the recursively updated one; on convergence the true residual B - H X is
computed, and if it misses the tolerance the method restarts from X with a
fresh shadow block (the recursion drifts from the true residual in finite
precision).
"""
from __future__ import annotations

import numpy as np

from . import Hierarchy, apply_fine, npts


def _apply(hier: Hierarchy, X):
    """H X for a block [s][N] (the unshifted operator, eq:LinearSystem)."""
    return apply_fine(hier.g, hier._m, hier._gamma, hier.omega, 0.0, X)


def block_bicgstab(hier: Hierarchy, B, tol=1e-6, maxcycles=1000, X0=None, prec=True, hist=False):
    """Block BiCGSTAB on the whole block B [s][N] (columns are rows of the
    array). prec: apply the hierarchy's cycle as right preconditioner (it
    must be stationary: LU or relaxation-only coarsest solve), else the
    identity. Returns (X, cycles, relres, converged[, residual history]);
    `cycles` counts preconditioner applications, two per iteration, and the
    history holds max_c ||r_c|| / ||b_c|| of the recursive residual after
    each iteration."""
    B = np.ascontiguousarray(B, dtype=np.complex128).reshape(-1, npts(hier.g))
    X = np.zeros_like(B) if X0 is None else np.array(X0, dtype=np.complex128).reshape(B.shape)
    bn = np.linalg.norm(B, axis=1)
    zero = bn == 0
    if zero.any():
        # a zero right-hand side is solved by zero; the block method runs on
        # the others (a zero column would make Rt^H V singular)
        out = list(block_bicgstab(hier, B[~zero], tol, maxcycles, None if X0 is None else X[~zero], prec, True))
        Xa = np.zeros_like(B)
        Xa[~zero] = out[0]
        rr = np.zeros(B.shape[0])
        rr[~zero] = out[2]
        res = (Xa, out[1], rr, out[3])
        return res + (out[4],) if hist else res
    bn_safe = np.where(bn > 0, bn, 1.0)
    prec_apply = hier.vcycle if prec else (lambda Y: np.array(Y, copy=True))
    cycles = 0
    history = []

    def relres_true():
        R = B - _apply(hier, X)
        return R, np.where(bn > 0, np.linalg.norm(R, axis=1) / bn_safe, 0.0)

    R, rr = relres_true()
    converged = bool(np.all(rr <= tol))
    while not converged and cycles < maxcycles:
        # (re)start: shadow block and first direction from the current residual
        Rt = R.copy()
        P = R.copy()
        while cycles < maxcycles:
            # matrices are stored with the block index first: column c of the
            # paper's N x s block is row c here, so Rt^H V is Rt.conj() @ V.T
            Phat = prec_apply(P)
            V = _apply(hier, Phat)
            cycles += 1
            A = Rt.conj() @ V.T                  # s x s: (Rt^H V)[a][c]
            try:
                alpha = np.linalg.solve(A, Rt.conj() @ R.T)
            except np.linalg.LinAlgError:
                break                            # breakdown: restart
            S = R - alpha.T @ V                  # R - V alpha
            Shat = prec_apply(S)
            T = _apply(hier, Shat)
            cycles += 1
            tt = np.vdot(T, T).real
            omega = np.vdot(T, S) / tt if tt > 0 else 0.0
            X = X + alpha.T @ Phat + omega * Shat
            R = S - omega * T
            est = np.where(bn > 0, np.linalg.norm(R, axis=1) / bn_safe, 0.0)
            history.append(float(est.max()))
            if np.all(est <= tol) or omega == 0.0:
                break
            beta = -np.linalg.solve(A, Rt.conj() @ T.T)
            P = R + beta.T @ (P - omega * V)
        R, rr = relres_true()
        converged = bool(np.all(rr <= tol))
    out = (X, cycles, rr, converged)
    if hist:
        out = out + (np.array(history),)
    return out
