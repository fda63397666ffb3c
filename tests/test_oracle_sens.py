"""Pins of the oracle's adjoint solve, sensitivity products and 16-bit field
storage (oracle/sens.py), each against something other than its formula:

  - J dm equals the central finite difference of the solution in the model,
    (u(m + e dm) - u(m - e dm)) / 2e, from two independent oracle solves;
  - the adjoint identity Re <w, J dm> = <Re J^H w, dm> and, for the adjoint
    solve, <H^-H w, q> = <w, H^-1 q>;
  - 16-bit storage: the largest entry of a column is stored as +-1 exactly,
    every entry is within half a unit in the last place of FP16 (plus the
    FP32 rounding taken first) of its scaled value, the round trip is within
    2^-11 of the column's scale, and a zero column stays zero.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import sens

RNG = np.random.default_rng(4242)


_SETUP = []


@pytest.fixture(scope="module")
def setup():
    return setup_problem()


def setup_problem():
    """The pins' 2D problem, its fields and a model perturbation (built once)."""
    if _SETUP:
        return _SETUP[0]
    p = synth.gradient_2d(n=48, nsrc=(2,), levels=3)
    g = oracle.grid(p.dim, p.n, p.h)
    h = oracle.Hierarchy(g, p.m, p.gamma, p.omega, p.shift, 3)
    U = sens.solve(h, p.Q, tol=1e-12)
    # a smooth real model perturbation
    x = np.linspace(0, 1, p.n[0] - 1)
    dm = (np.sin(3 * np.pi * x)[:, None] * np.cos(2 * np.pi * x)[None, :]).ravel() * 0.05 * p.m.max()
    _SETUP.append((p, g, h, U, dm))
    return _SETUP[0]


def test_jvp_equals_central_difference(setup):
    p, g, h, U, dm = setup
    J = sens.jvp(h, U, dm, tol=1e-12)
    eps = 1e-4
    up = sens.solve(oracle.Hierarchy(g, p.m.ravel() + eps * dm, p.gamma, p.omega, p.shift, 3), p.Q, tol=1e-12)
    um = sens.solve(oracle.Hierarchy(g, p.m.ravel() - eps * dm, p.gamma, p.omega, p.shift, 3), p.Q, tol=1e-12)
    fd = (up - um) / (2 * eps)
    assert np.linalg.norm(J - fd) <= 1e-5 * np.linalg.norm(fd), np.linalg.norm(J - fd) / np.linalg.norm(fd)


def test_adjoint_identities(setup):
    p, g, h, U, dm = setup
    W = RNG.standard_normal(U.shape) + 1j * RNG.standard_normal(U.shape)
    J = sens.jvp(h, U, dm, tol=1e-12)
    lhs = np.real(np.vdot(W, J))
    rhs = np.dot(sens.jtvp(h, U, W, tol=1e-12), dm)
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs), (lhs, rhs)
    Y = sens.solve(h, W, tol=1e-12, op="A")
    X = sens.solve(h, p.Q, tol=1e-12)
    for s in range(W.shape[0]):
        a, b = np.vdot(Y[s], p.Q[s]), np.vdot(W[s], X[s])
        assert abs(a - b) <= 1e-9 * abs(b)


def test_pack16_bounds():
    U = (RNG.standard_normal((3, 5000)) + 1j * RNG.standard_normal((3, 5000))) * np.array([1e5, 1e-3, 7.0])[:, None]
    h, s = sens.pack16(U)
    assert h.dtype == np.float16 and h.shape == (3, 5000, 2)
    for c in range(3):
        assert np.max(np.abs(h[c].astype(np.float64))) == 1.0
    V = U / s[:, None]
    for part, k in ((V.real, 0), (V.imag, 1)):
        err = np.abs(h[..., k].astype(np.float64) - part)
        ulp = np.spacing(np.maximum(np.abs(part), 2.0 ** -14).astype(np.float16)).astype(np.float64)
        # half a unit of FP16, plus the FP32 rounding taken first
        assert np.all(err <= 0.5 * ulp + 2.0 ** -24 * np.abs(part))
    W = sens.unpack16(h, s)
    assert np.max(np.abs(W - U) / s[:, None]) <= 2.0 ** -11
    Z = np.zeros((1, 7), np.complex128)
    hz, sz = sens.pack16(Z)
    assert sz[0] == 1.0 and np.all(hz == 0)
