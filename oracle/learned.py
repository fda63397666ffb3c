"""Oracle of the learned coarsest-grid correction as the multigrid cycle
applies it, and of the Adam update that trains it (test infrastructure only:
only tests/, the smoke check and the benchmark's CPU baseline use oracle/;
the solver library never imports or calls it).

The paper names a cheaper stationary inexact solver of the coarsest grid as
future work (end of section 5.3 and the conclusions) and gives no design;
the composition below is this project's reading of it, written out in plain
FP64 numpy around the oracle's pinned primitives (the coarsest Galerkin
stencil, its operator, fixed-step GMRES from zero, the U-Net forward pass):

  1. per column s of the coarsest right-hand side f: rms_s = ||f_s||_2 /
     sqrt(Nc) over the Nc unknowns of the coarsest grid;
  2. the network input on a D^3 volume (unknown (x, y, z) at voxel (x, y, z),
     zeros elsewhere), four channels per voxel: Re and Im of f_s / rms_s, Re
     and Im of H^2 times the centre coefficient of the coarsest Galerkin
     stencil (H the coarsest mesh width);
  3. out = network(input), two channels;
  4. e_s = H^2 rms_s (out_0 + i out_1) on the unknowns (0 for a zero column);
  5. if any output of the block is not finite or beyond 1e4 in magnitude,
     the whole block's e is replaced by max(k, 20) GMRES steps from zero
     (the fallback);
  6. otherwise, `restarts` times: r = f - M_c e, e += GMRES_k(r) from zero
     (k = 0: the network alone).

Adam follows Kingma & Ba (2015), Algorithm 1: with gradient g_t at step t,
m_t = b1 m + (1 - b1) g_t, v_t = b2 v + (1 - b2) g_t^2,
theta -= lr (m_t / (1 - b1^t)) / (sqrt(v_t / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

from . import Hierarchy, apply_stencil, npts


def coarsest_view(hier: Hierarchy):
    """(grid, stencil [Nc][27], H^2) of the hierarchy's coarsest level."""
    L = hier.levels - 1
    g = hier.level_grid(L)
    return g, hier.stencil(L), g.h[0] * g.h[0]


def net_input(hier: Hierarchy, F, D: int) -> np.ndarray:
    """Steps 1-2: the network input [B, D, D, D, 4] (channels last, axis 0 of
    the grid fastest, i.e. numpy index [b, z, y, x, c]) and rms [B]."""
    g, st, H2 = coarsest_view(hier)
    nx, ny, nz = g.nu[0], g.nu[1], g.nu[2]
    Nc = npts(g)
    F = np.asarray(F, dtype=np.complex128).reshape(-1, Nc)
    B = F.shape[0]
    rms = np.sqrt(np.sum(np.abs(F) ** 2, axis=1) / Nc)
    x = np.zeros((B, D, D, D, 4))
    centre = (H2 * st[:, 13]).reshape(nz, ny, nx)
    for b in range(B):
        fs = F[b] / rms[b] if rms[b] > 0 else np.zeros(Nc, np.complex128)
        fs = fs.reshape(nz, ny, nx)
        x[b, :nz, :ny, :nx, 0] = fs.real
        x[b, :nz, :ny, :nx, 1] = fs.imag
        x[b, :nz, :ny, :nx, 2] = centre.real
        x[b, :nz, :ny, :nx, 3] = centre.imag
    return x, rms


def learned_coarse_solve(hier_gmres: Hierarchy, F, D: int, net, k: int, restarts: int = 1):
    """The learned coarsest solve of a block F [B][Nc] (steps 1-6).

    hier_gmres: an oracle Hierarchy of the problem whose coarse solve is
    k' = k steps of GMRES from zero with one cycle (coarse="gmres",
    coarse_iters=max(k, 1)); its coarse_solve is the pinned GMRES_k.
    net: callable mapping an input [B, D, D, D, 4] to [B, D, D, D, 2].
    Returns (E [B][Nc], fallback: bool)."""
    g, st, H2 = coarsest_view(hier_gmres)
    nx, ny, nz = g.nu[0], g.nu[1], g.nu[2]
    Nc = npts(g)
    F = np.asarray(F, dtype=np.complex128).reshape(-1, Nc)
    x, rms = net_input(hier_gmres, F, D)
    out = np.asarray(net(x), dtype=np.float64)
    if not (np.all(np.isfinite(out)) and np.abs(out).max(initial=0.0) <= 1e4):
        nu1, nu2, w = hier_gmres._keep
        fb = Hierarchy(hier_gmres.g, hier_gmres._m, hier_gmres._gamma, hier_gmres.omega, hier_gmres.beta,
                       hier_gmres.levels, nu_pre=nu1, nu_post=nu2, wjac=w, coarse="gmres",
                       coarse_iters=max(k, 20))
        return fb.coarse_solve(F), True
    E = np.empty_like(F)
    for b in range(F.shape[0]):
        o = out[b, :nz, :ny, :nx, :]
        E[b] = (H2 * rms[b]) * (o[..., 0] + 1j * o[..., 1]).reshape(Nc)
    if k > 0:
        for _ in range(restarts):
            R = F - apply_stencil(g, st, E)
            E = E + hier_gmres.coarse_solve(R)
    return E, False


def adam(theta0, grads, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Parameters after Adam steps t = 1..len(grads) from theta0 with zero
    moments (Kingma & Ba, Algorithm 1), in FP64. Returns the list of
    parameter vectors after each step."""
    theta = np.asarray(theta0, dtype=np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    out = []
    for t, g in enumerate(grads, start=1):
        g = np.asarray(g, dtype=np.float64)
        m = b1 * m + (1.0 - b1) * g
        v = b2 * v + (1.0 - b2) * g * g
        mhat = m / (1.0 - b1 ** t)
        vhat = v / (1.0 - b2 ** t)
        theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
        out.append(theta.copy())
    return out
