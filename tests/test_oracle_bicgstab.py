"""Pins of the oracle's block BiCGSTAB (oracle/bicgstab.py), each against
something other than the code itself:

  - one right-hand side without preconditioner: the iterates are those of
    scipy.sparse.linalg.bicgstab (a library implementation of van der
    Vorst's method, to which the block method reduces for s = 1);
  - tiny grids, dense reference: a block of right-hand sides solved to 1e-12
    equals numpy.linalg.solve of the assembled operator;
  - manufactured solution with the stationary cycle (banded-LU coarsest) as
    right preconditioner returns the chosen solution, and agrees with the
    oracle's block FGMRES solution;
  - a zero column is solved by zero.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle import bicgstab as ob

RNG = np.random.default_rng(515)


def hier_for(p, levels=3, coarse="lu"):
    return oracle.Hierarchy(oracle.grid(p.dim, p.n, p.h), p.m, p.gamma, p.omega, p.shift, levels, coarse=coarse)


@pytest.mark.parametrize("omega_scale,iters,rtol", [(1.0, (1, 3, 5), 1e-12), (0.1, (4, 8, 12), 1e-10)])
def test_single_rhs_unpreconditioned_matches_scipy(omega_scale, iters, rtol):
    """On the indefinite Helmholtz operator the two implementations agree to
    rounding for the first iterations (later the unpreconditioned method
    amplifies rounding differences exponentially: 1e-16 at 5, 1e-9 at 8,
    1e-1 at 12 iterations); at a tenth of the frequency, where the method
    is stable, for 12 iterations."""
    p = synth.gradient_2d(n=32, nsrc=(1,), levels=2)
    om = p.omega * omega_scale
    h = oracle.Hierarchy(oracle.grid(p.dim, p.n, p.h), p.m, p.gamma, om, p.shift, 2)
    g = h.g
    A = spla.LinearOperator((p.N, p.N), dtype=np.complex128,
                            matvec=lambda x: oracle.apply_fine(g, p.m, p.gamma, om, 0.0, x[None, :])[0])
    b = p.Q[0] + 0.5 * (RNG.standard_normal(p.N) + 1j * RNG.standard_normal(p.N)) * np.abs(p.Q[0]).max()
    xs = []
    spla.bicgstab(A, b, rtol=1e-30, maxiter=max(iters), callback=lambda xk: xs.append(xk.copy()))
    for it in iters:
        X, cyc, rr, conv = ob.block_bicgstab(h, b[None, :], tol=1e-30, maxcycles=2 * it, prec=False)
        assert cyc == 2 * it
        ref = xs[it - 1]
        assert np.linalg.norm(X[0] - ref) <= rtol * np.linalg.norm(ref), it


@pytest.mark.parametrize("dim,n", [(2, 8), (3, 6)])
def test_block_solve_equals_dense_solve(dim, n):
    if dim == 2:
        p = synth.gradient_2d(n=n, nsrc=(1,), levels=2)
    else:
        p = synth.layered_3d(n=n, nsrc=(1, 1), levels=2, seed=2)
    h = hier_for(p, 2)
    g = h.g
    Hd = oracle.apply_fine(g, p.m, p.gamma, p.omega, 0.0, np.eye(p.N, dtype=np.complex128)).T
    B = RNG.standard_normal((3, p.N)) + 1j * RNG.standard_normal((3, p.N))
    X, cyc, rr, conv = ob.block_bicgstab(h, B, tol=1e-12, maxcycles=4000, prec=False)
    ref = np.linalg.solve(Hd, B.T).T
    assert conv and np.linalg.norm(X - ref) <= 1e-9 * np.linalg.norm(ref)


@pytest.mark.parametrize("dim,n,levels", [(2, 48, 3), (3, 24, 3)])
def test_manufactured_solution_with_stationary_cycle(dim, n, levels):
    if dim == 2:
        p = synth.gradient_2d(n=n, nsrc=(2,), levels=levels)
    else:
        p = synth.layered_3d(n=n, nsrc=(2, 1), levels=levels, seed=2)
    h = hier_for(p, levels)
    Xs = RNG.standard_normal((4, p.N)) + 1j * RNG.standard_normal((4, p.N))
    B = oracle.apply_fine(h.g, p.m, p.gamma, p.omega, 0.0, Xs)
    X, cyc, rr, conv = ob.block_bicgstab(h, B, tol=1e-11, maxcycles=2000)
    assert conv and rr.max() <= 1e-11
    assert np.linalg.norm(X - Xs) <= 1e-7 * np.linalg.norm(Xs)
    Xf, it, rf, cf = h.fgmres(B, tol=1e-11, restart=5, maxit=2000)
    assert cf and np.linalg.norm(X - Xf) <= 1e-7 * np.linalg.norm(Xf)


def test_zero_column_is_solved_by_zero():
    p = synth.gradient_2d(n=32, nsrc=(3,), levels=3)
    h = hier_for(p, 3)
    B = p.Q.copy()
    B[1] = 0.0
    X, cyc, rr, conv = ob.block_bicgstab(h, B, tol=1e-8, maxcycles=500)
    assert conv and np.all(X[1] == 0) and rr[1] == 0.0 and rr.max() <= 1e-8
