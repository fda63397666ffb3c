"""Pins of the oracle's learned coarsest solve and Adam update
(oracle/learned.py), each against something other than the composition
itself:

  - a network that outputs zero reduces the learned solve to the oracle's
    restarted GMRES from zero (a C primitive pinned elsewhere);
  - a network that outputs a constant, with no GMRES steps, gives the closed
    form e = H^2 rms(f) (c0 + i c1) on every unknown;
  - probe networks that copy input channels to the output give the closed
    forms H^2 f (channels 0, 1) and H^4 diag(M_c) (channels 2, 3);
  - a network that outputs the exact coarsest solution (normalised) gives the
    banded-LU solve, also after GMRES steps (GMRES starts from the guess);
  - the real U-Net composition is positively homogeneous of degree 1;
  - an output beyond the bound switches to max(k, 20) GMRES steps from zero;
  - Adam reproduces a two-step case worked out by hand
    (tests/golden/adam_two_steps.txt) and the first-step identity
    theta1 = theta0 - lr g / (|g| + eps) of the bias-corrected moments.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import learned as ol

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
RNG = np.random.default_rng(31)


@pytest.fixture(scope="module")
def prob():
    return synth.layered_3d(n=32, nsrc=(2, 2), levels=3, seed=2)


def hier(p, coarse, k=8, restarts=1):
    return oracle.Hierarchy(oracle.grid(p.dim, p.n, p.h), p.m, p.gamma, p.omega, p.shift, 3, coarse=coarse,
                            coarse_iters=k, coarse_restarts=restarts)


def coarse_rhs(h, B=3):
    g = h.level_grid(h.levels - 1)
    F = RNG.standard_normal((B, oracle.npts(g))) + 1j * RNG.standard_normal((B, oracle.npts(g)))
    F[1] = 0.0  # a zero column stays zero
    return g, F


def edge(g):
    return (max(g.nu[0], g.nu[1], g.nu[2]) + 3) // 4 * 4


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("k,restarts", [(4, 1), (8, 2)])
def test_zero_network_is_restarted_gmres_from_zero(prob, k, restarts):
    h = hier(prob, "gmres", k)
    g, F = coarse_rhs(h)
    E, fb = ol.learned_coarse_solve(h, F, edge(g), lambda x: np.zeros(x.shape[:4] + (2,)), k, restarts)
    ref = hier(prob, "gmres", k, restarts).coarse_solve(F)
    assert not fb and rel(E, ref) <= 1e-13


def test_constant_network_closed_form(prob):
    h = hier(prob, "gmres", 4)
    g, F = coarse_rhs(h)
    c = (0.37, -1.25)

    def net(x):
        out = np.zeros(x.shape[:4] + (2,))
        out[..., 0], out[..., 1] = c
        return out
    E, _ = ol.learned_coarse_solve(h, F, edge(g), net, 0)
    H2 = g.h[0] ** 2
    rms = np.sqrt(np.mean(np.abs(F) ** 2, axis=1))
    ref = (H2 * rms)[:, None] * (c[0] + 1j * c[1]) * np.ones_like(F)
    assert np.allclose(E, ref, rtol=1e-15, atol=0.0)
    assert np.all(E[1] == 0)


def test_probe_networks_see_the_stated_channels(prob):
    h = hier(prob, "gmres", 4)
    g, F = coarse_rhs(h)
    H2 = g.h[0] ** 2
    E01, _ = ol.learned_coarse_solve(h, F, edge(g), lambda x: x[..., 0:2].copy(), 0)
    assert rel(E01, H2 * F) <= 1e-15
    E23, _ = ol.learned_coarse_solve(h, F, edge(g), lambda x: x[..., 2:4].copy(), 0)
    st = h.stencil(h.levels - 1)
    rms = np.sqrt(np.mean(np.abs(F) ** 2, axis=1))
    ref = (H2 * rms)[:, None] * (H2 * st[:, 13])[None, :]
    assert rel(E23, ref) <= 1e-15 and np.all(E23[1] == 0)


@pytest.mark.parametrize("k,restarts", [(0, 1), (8, 2)])
def test_perfect_network_gives_the_exact_solve(prob, k, restarts):
    h = hier(prob, "gmres", max(k, 1))
    g, F = coarse_rhs(h)
    exact = hier(prob, "lu").coarse_solve(F)
    nx, ny, nz = g.nu[0], g.nu[1], g.nu[2]
    H2 = g.h[0] ** 2
    rms = np.sqrt(np.mean(np.abs(F) ** 2, axis=1))
    D = edge(g)

    def net(x):
        out = np.zeros(x.shape[:4] + (2,))
        for b in range(x.shape[0]):
            if rms[b] > 0:
                e = (exact[b] / (H2 * rms[b])).reshape(nz, ny, nx)
                out[b, :nz, :ny, :nx, 0], out[b, :nz, :ny, :nx, 1] = e.real, e.imag
        return out
    E, _ = ol.learned_coarse_solve(h, F, D, net, k, restarts)
    assert rel(E, exact) <= 1e-10


def test_unet_composition_is_homogeneous(prob):
    h = hier(prob, "gmres", 4)
    g, F = coarse_rhs(h)
    prm = RNG.standard_normal(oracle.unet_nparams()) * 0.05

    def net(x):
        return oracle.unet_forward(prm, x)
    E, _ = ol.learned_coarse_solve(h, F, edge(g), net, 4, 2)
    E2, _ = ol.learned_coarse_solve(h, 3.7 * F, edge(g), net, 4, 2)
    assert rel(E2, 3.7 * E) <= 1e-12


def test_fallback_on_nonfinite_or_huge_output(prob):
    h = hier(prob, "gmres", 4)
    g, F = coarse_rhs(h)
    ref = hier(prob, "gmres", 20).coarse_solve(F)
    for bad in (np.nan, 2e4):
        E, fb = ol.learned_coarse_solve(h, F, edge(g), lambda x: np.full(x.shape[:4] + (2,), bad), 4)
        assert fb and rel(E, ref) <= 1e-14


def test_adam_two_steps_worked_by_hand():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "adam_two_steps.txt")) if ln.strip() and ln[0] != "#"]
    grads = [np.array([float(r[1])]) for r in rows]
    out = ol.adam(np.array([1.0]), grads, lr=0.1)
    for r, th in zip(rows, out):
        assert abs(th[0] - float(r[2])) <= 1e-15, (r, th)


def test_adam_first_step_identity():
    g = RNG.standard_normal(1000) * np.logspace(-6, 2, 1000)
    th0 = RNG.standard_normal(1000)
    (th1,) = ol.adam(th0, [g], lr=3e-3)
    assert np.allclose(th1, th0 - 3e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
