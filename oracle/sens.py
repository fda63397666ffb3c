"""Oracle of the transposed and adjoint solves, the sensitivity products of
full waveform inversion and the 16-bit storage of fields (test
infrastructure only: only tests/, the smoke check and the benchmark's CPU
baseline use oracle/; the solver library never imports or calls it).

Sensitivities (the Helmholtz forward problem and its sensitivities,
eq:fwisens). With H(m) u = q, H = -Lap_h - omega^2 diag(m (1 - i gamma))
(the paper's operator with q negated), differentiating in the real model m
gives H du = omega^2 diag((1 - i gamma) u) dm, so

    J dm   = omega^2 H^-1 ((1 - i gamma) u . dm),
    J^H w  = omega^2 conj((1 - i gamma) u) . H^-H w,

and the gradient of a real misfit in m takes Re(J^H w), summed over the
sources. H is complex symmetric (H^T = H: a symmetric stencil plus a
diagonal), so the transposed system is the system itself (the paper's remark
that the transposed problem reuses the hierarchy), and the adjoint solve is
H^-H w = conj(H^-1 conj(w)).

16-bit fields: the paper stores fields in a 16-bit floating point format
(32 bits per complex unknown). Here each source's field is divided by its
largest real or imaginary magnitude s_c (kept in FP64), rounded to FP32 and
then to IEEE half precision (round to nearest even): u ~ s_c * half(u / s_c).
"""
from __future__ import annotations

import numpy as np

from . import Hierarchy, apply_fine, npts


def solve(hier: Hierarchy, B, tol=1e-10, op="H"):
    """H X = B (op "H"), H^T X = B ("T"; the same system) or H^H X = B ("A",
    the adjoint: conj of the solve of conj(B)), by the oracle's block
    FGMRES(5) with its cycle to `tol`. Returns X [s][N]."""
    B = np.ascontiguousarray(B, dtype=np.complex128).reshape(-1, npts(hier.g))
    if op == "A":
        return np.conj(solve(hier, np.conj(B), tol, "H"))
    X, it, rr, conv = hier.fgmres(B, tol=tol, restart=5, maxit=4000)
    if not conv:
        raise RuntimeError("oracle solve did not converge")
    return X


def dH_dm_factor(hier: Hierarchy) -> np.ndarray:
    """omega^2 (1 - i gamma) per unknown: H(m + dm) - H(m) = -diag(this * dm)."""
    return hier.omega ** 2 * (1.0 - 1j * hier._gamma)


def jvp(hier: Hierarchy, U, dm, tol=1e-10):
    """J dm for each field u_s (rows of U): omega^2 H^-1 ((1 - i gamma) u_s dm)."""
    U = np.ascontiguousarray(U, dtype=np.complex128).reshape(-1, npts(hier.g))
    rhs = dH_dm_factor(hier)[None, :] * U * np.asarray(dm, dtype=np.float64).ravel()[None, :]
    return solve(hier, rhs, tol, "H")


def jtvp(hier: Hierarchy, U, W, tol=1e-10):
    """Re sum_s J_s^H w_s: omega^2 Re sum_s conj((1 - i gamma) u_s) H^-H w_s."""
    U = np.ascontiguousarray(U, dtype=np.complex128).reshape(-1, npts(hier.g))
    Y = solve(hier, W, tol, "A")
    return np.real(np.sum(np.conj(dH_dm_factor(hier)[None, :] * U) * Y, axis=0))


def pack16(U):
    """16-bit storage of fields: (half [s][N][2] of re, im of u / s_c, and
    s_c [s] = the column's largest |re| or |im|; 1 for a zero column)."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    s = np.max(np.maximum(np.abs(U.real), np.abs(U.imag)), axis=1)
    s = np.where(s > 0, s, 1.0)
    vr = U.real / s[:, None]  # real and imaginary parts divided separately, in FP64
    vi = U.imag / s[:, None]
    h = np.stack([vr.astype(np.float32).astype(np.float16), vi.astype(np.float32).astype(np.float16)], -1)
    return h, s


def unpack16(h, s):
    """Fields from their 16-bit storage: s_c * (re + i im)."""
    h = np.asarray(h, dtype=np.float16).astype(np.float64)
    return (h[..., 0] + 1j * h[..., 1]) * np.asarray(s, dtype=np.float64)[:, None]
