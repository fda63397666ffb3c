"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Every comparison is element by element on the same seeded inputs, at sizes
that span several tiles and a ragged tail. Tolerances (relative, 2-norm or
max-norm as stated) follow from the arithmetic:
  - FP64 operator apply: a handful of roundings per entry -> 1e-13;
  - FP64 Galerkin stencils: sums of <= 729 products -> 1e-12;
  - FP64 coarsest solve (explicit inverse vs banded LU): kappa(M_c) * eps,
    kappa of the shifted coarsest operator is below 1e3 here -> 1e-10;
  - FP64 V-cycle: a fixed linear map; the divergent coarse smoothing
    amplifies rounding by at most ~1e2 -> 1e-9;
  - solves: every column reaches the FP64 relative residual tol (checked by
    the oracle's own operator) and the error against the oracle's solution
    (solved to 1e-10) is bounded by kappa * tol; the stated bound 1e-5 is
    checked at a GPU tolerance of 1e-8 (see the error-vs-residual reading).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pk = pytest.importorskip("paper_1607_00968_amd")

RNG = np.random.default_rng(77)


def crand(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def small_problem(dim, n, levels, seed=5, nsrc=None):
    if dim == 2:
        p = synth.gradient_2d(n=n, nsrc=nsrc or (3,), levels=levels)
    else:
        p = synth.layered_3d(n=n, nsrc=nsrc or (2, 2), levels=levels, seed=2)
    return p


def setup_both(p, levels, precision="fp64", coarse="lu", coarse_iters=20, coarse_restarts=1):
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, shift=p.shift, levels=levels,
                       precision=precision, coarse=coarse, coarse_iters=coarse_iters,
                       coarse_restarts=coarse_restarts)
    ho = oracle.Hierarchy(oracle.grid(p.dim, p.n, p.h), p.m, p.gamma, p.omega, p.shift, levels,
                          coarse="gmres" if coarse == "gmres" else "lu", coarse_iters=coarse_iters,
                          coarse_restarts=coarse_restarts)
    return hd, ho


GRIDS = [(2, 24, 3), (2, 40, 2), (3, 16, 3), (3, 24, 2)]


@pytest.mark.parametrize("dim,n,levels", GRIDS)
@pytest.mark.parametrize("nrhs", [1, 3, 8])
def test_apply_matches_oracle(dim, n, levels, nrhs):
    p = small_problem(dim, n, levels)
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, levels=levels)
    g = oracle.grid(p.dim, p.n, p.h)
    X = crand(nrhs, p.N)
    for shifted, beta in ((False, 0.0), (True, p.shift)):
        Y = torch.empty((nrhs, p.N), dtype=torch.complex128, device="cuda")
        pk.helm_apply(hd, dev(X), Y, shifted=shifted)
        ref = oracle.apply_fine(g, p.m, p.gamma, p.omega, beta, X)
        assert np.abs(host(Y) - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("dim,n,levels", [(2, 32, 3), (3, 16, 3), (3, 32, 3)])
def test_galerkin_stencils_match_oracle(dim, n, levels):
    p = small_problem(dim, n, levels)
    hd, ho = setup_both(p, levels)
    for l in range(1, levels):
        st = pk.helm_level_stencil(hd, l)
        ref = ho.stencil(l)
        if dim == 2:
            ref = ref[:, 9:18]  # oz = 0 slab of the oracle's 27-entry form
        assert np.abs(st - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("dim,n,levels", [(2, 32, 3), (3, 16, 3), (3, 16, 2)])
def test_coarse_lu_solve_matches_oracle(dim, n, levels):
    p = small_problem(dim, n, levels)
    hd, ho = setup_both(p, levels)
    nu = pk.helm_level_dims(hd, levels - 1)
    Nc = int(np.prod(nu))
    F = crand(5, Nc)
    E = torch.empty((5, Nc), dtype=torch.complex128, device="cuda")
    pk.helm_coarse_solve(hd, dev(F), E)
    assert rel(host(E), ho.coarse_solve(F)) <= 1e-10


@pytest.mark.parametrize("k,restarts", [(4, 1), (20, 1), (4, 3)])
def test_coarse_gmres_matches_oracle(k, restarts):
    p = small_problem(3, 32, 3)
    hd, ho = setup_both(p, 3, coarse="gmres", coarse_iters=k, coarse_restarts=restarts)
    Nc = int(np.prod(pk.helm_level_dims(hd, 2)))
    F = crand(6, Nc)
    E = torch.empty((6, Nc), dtype=torch.complex128, device="cuda")
    pk.helm_coarse_solve(hd, dev(F), E)
    assert rel(host(E), ho.coarse_solve(F)) <= 1e-9


def test_vcycle_fp64_restarted_gmres_coarsest_matches_oracle():
    p = small_problem(3, 32, 3)
    hd, ho = setup_both(p, 3, coarse="gmres", coarse_iters=6, coarse_restarts=2)
    F = crand(3, p.N)
    Z = torch.empty((3, p.N), dtype=torch.complex128, device="cuda")
    pk.helm_precond(hd, dev(F), Z)
    assert rel(host(Z), ho.vcycle(F)) <= 1e-9


@pytest.mark.parametrize("dim,n,levels,coarse", [(2, 32, 3, "lu"), (3, 16, 3, "lu"), (3, 32, 3, "gmres"),
                                                 (2, 48, 4, "lu")])
@pytest.mark.parametrize("nrhs", [1, 5])
def test_vcycle_fp64_matches_oracle(dim, n, levels, coarse, nrhs):
    p = small_problem(dim, n, levels)
    hd, ho = setup_both(p, levels, coarse=coarse)
    F = crand(nrhs, p.N)
    Z = torch.empty((nrhs, p.N), dtype=torch.complex128, device="cuda")
    pk.helm_precond(hd, dev(F), Z)
    assert rel(host(Z), ho.vcycle(F)) <= 1e-9


@pytest.mark.parametrize("dim,n,levels,coarse", [(2, 32, 3, "lu"), (3, 32, 3, "gmres"), (2, 64, 3, "lu"),
                                                 (3, 48, 3, "gmres")])
def test_vcycle_mixed_close_to_oracle(dim, n, levels, coarse):
    """FP32 cycle with BF16 fields below the finest level against the FP64
    oracle's cycle, per column. The fields of the coarse levels are stored in
    BF16 (round to nearest even: a relative error of at most 2^-9 per value),
    and the coarse correction carries that error into the output; the FP32
    arithmetic adds about 1e-7. Measured 1.1e-3 to 1.9e-3 (0.6 to 0.95 BF16
    units) over these cases and seeds; the bound is two BF16 units, 2^-8."""
    p = small_problem(dim, n, levels)
    hd, ho = setup_both(p, levels, precision="mixed", coarse=coarse)
    F = crand(4, p.N)
    Z = torch.empty((4, p.N), dtype=torch.complex128, device="cuda")
    pk.helm_precond(hd, dev(F), Z)
    Zh, Zo = host(Z), ho.vcycle(F)
    for c in range(4):
        assert rel(Zh[c], Zo[c]) <= 2.0 ** -8, (c, rel(Zh[c], Zo[c]))


def check_solution(p, U, tol_res, Uref=None, err_tol=None):
    g = oracle.grid(p.dim, p.n, p.h)
    R = p.Q - oracle.apply_fine(g, p.m, p.gamma, p.omega, 0.0, U)
    rr = np.linalg.norm(R, axis=1) / np.linalg.norm(p.Q, axis=1)
    assert rr.max() <= tol_res, rr
    if Uref is not None:
        err = np.linalg.norm(U - Uref, axis=1) / np.linalg.norm(Uref, axis=1)
        assert err.max() <= err_tol, err
    return rr


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("block_size", [4, 1])
def test_solve_2d_128_gradient(precision, block_size):
    p = synth.gradient_2d()  # 2D 128^2, 4 sources, 3 levels, FGMRES(10)
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, levels=3, precision=precision)
    Q = dev(p.Q)
    U = torch.zeros_like(Q)
    info = pk.helm_solve_block(hd, Q, U, tol=1e-8, restart=10, max_cycles=2000, block_size=block_size)
    assert info["converged_all"], info
    ho = oracle.setup_problem(p, levels=3)
    Xo, it, rr, conv = ho.fgmres(p.Q, tol=1e-10, restart=10, maxit=3000)
    assert conv
    check_solution(p, host(U), 1e-8, Xo, 1e-5)
    # the library's own FP64 residual agrees with the oracle's
    assert np.allclose(pk.helm_residual(hd, Q, U), info["relres"], rtol=1e-6, atol=1e-14)


@pytest.mark.parametrize("precision,coarse", [("fp64", "lu"), ("mixed", "gmres")])
def test_solve_3d_small(precision, coarse):
    p = synth.layered_3d(n=32, nsrc=(3, 2), levels=3, seed=2)  # ragged: 6 sources
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, levels=3, precision=precision, coarse=coarse)
    Q = dev(p.Q)
    U = torch.zeros_like(Q)
    info = pk.helm_solve_block(hd, Q, U, tol=1e-6, restart=5, max_cycles=2000, block_size=1)
    assert info["converged_all"], info
    check_solution(p, host(U), 1e-6)
    assert (info["relres"] <= 1e-6).all()


def test_solve_tracks_oracle_cycle_count_fp64():
    """Same algorithm, same stopping rule: FP64 cycle counts agree closely."""
    p = synth.gradient_2d(n=64, nsrc=(1,), levels=3)
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, levels=3)
    Q = dev(p.Q)
    U = torch.zeros_like(Q)
    info = pk.helm_solve_block(hd, Q, U, tol=1e-6, restart=10, max_cycles=2000, reorth=True)
    ho = oracle.setup_problem(p, levels=3)
    Xo, it, rr, conv = ho.fgmres(p.Q, tol=1e-6, restart=10, maxit=2000)
    assert abs(info["cycles"] - it) <= max(2, 0.02 * it), (info["cycles"], it)


def test_zero_column_converged_at_zero():
    p = synth.gradient_2d(n=32, nsrc=(3,), levels=3)
    Qn = p.Q.copy()
    Qn[1] = 0
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, levels=3)
    Q = dev(Qn)
    U = torch.zeros_like(Q)
    info = pk.helm_solve_block(hd, Q, U, tol=1e-7, restart=10, block_size=1)
    assert info["converged_all"]
    Uh = host(U)
    assert np.abs(Uh[1]).max() == 0.0 and info["relres"][1] == 0.0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_duplicate_and_dependent_sources_in_one_block(precision):
    """Rank-deficient blocks (the deflation of the block method): groups of
    3 holding a duplicate source ([q0, q1, q0]) and a combination
    ([q1, q0 + 2 q1, q0]) are solved: every column meets the tolerance by
    the oracle's FP64 operator, the duplicate columns agree to 1e-10, the
    combination equals the same combination of solutions to the solve's
    accuracy, and each column matches the oracle's deflated block FGMRES
    solution (tolerance 1e-10) within 1e-5 at a GPU tolerance of 1e-8.
    Block size 1 gives the same solutions."""
    p = synth.gradient_2d(n=32, nsrc=(2,), levels=3)
    q0, q1 = p.Q[0], p.Q[1]
    Qd = np.stack([q0, q1, q0, q1, q0 + 2 * q1, q0])
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, levels=3, precision=precision)
    Q = dev(Qd)
    U = torch.zeros_like(Q)
    info = pk.helm_solve_block(hd, Q, U, tol=1e-8, restart=10, block_size=3)
    assert info["converged_all"]
    Uh = host(U)
    assert np.isfinite(Uh).all()
    g = oracle.grid(p.dim, p.n, p.h)
    R = Qd - oracle.apply_fine(g, p.m, p.gamma, p.omega, 0.0, Uh)
    assert (np.linalg.norm(R, axis=1) / np.linalg.norm(Qd, axis=1)).max() <= 1e-8
    # within a group the duplicate keeps the same coefficients; across groups
    # (separate Krylov spaces) the solutions agree to the solve's accuracy
    assert rel(Uh[2], Uh[0]) < 1e-10
    assert rel(Uh[5], Uh[0]) < 1e-6 and rel(Uh[3], Uh[1]) < 1e-6
    assert rel(Uh[4], Uh[0] + 2 * Uh[1]) < 1e-6
    ho = oracle.setup_problem(p)
    Xo, it, rr, conv = ho.fgmres(Qd, tol=1e-10, restart=10, maxit=400)
    assert conv
    for c in range(6):
        assert rel(Uh[c], Xo[c]) < 1e-5, c
    U1 = torch.zeros_like(Q)
    info1 = pk.helm_solve_block(hd, Q, U1, tol=1e-8, restart=10, block_size=1)
    assert info1["converged_all"]
    Uh1 = host(U1)
    assert rel(Uh1[2], Uh1[0]) < 1e-12
    for c in range(6):
        assert rel(Uh[c], Uh1[c]) < 1e-5, c


_B64 = {}


def _block64_oracle(p, Qb):
    """The oracle's block FGMRES(5) solution of the 64-column block (computed
    once for the parametrised cases)."""
    if "X" not in _B64:
        Xo, it, rr, conv = oracle.setup_problem(p).fgmres(Qb, tol=1e-10, restart=5, maxit=400)
        assert conv
        _B64["X"] = Xo
    return _B64["X"]


@pytest.mark.parametrize("method,precision", [("fgmres", "fp64"), ("fgmres", "mixed"), ("bicgstab", "fp64")])
def test_block_of_64_columns(method, precision):
    """One block of 64 right-hand sides (the largest block size; the paper's
    tables go up to 64 sources): every column meets the tolerance by the
    oracle's FP64 operator and matches the oracle's block FGMRES solution
    (tolerance 1e-10, same block of 64) within 1e-5 at a GPU tolerance of
    1e-8."""
    p = synth.gradient_2d(n=64, nsrc=(2,), levels=3)
    rng = np.random.default_rng(64)
    Qb = rng.standard_normal((64, p.N)) + 1j * rng.standard_normal((64, p.N))
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, levels=3, precision=precision)
    Q = dev(Qb)
    U = torch.zeros_like(Q)
    info = pk.helm_solve_block(hd, Q, U, tol=1e-8, restart=5, block_size=64, method=method)
    assert info["converged_all"]
    Uh = host(U)
    g = oracle.grid(p.dim, p.n, p.h)
    R = Qb - oracle.apply_fine(g, p.m, p.gamma, p.omega, 0.0, Uh)
    assert (np.linalg.norm(R, axis=1) / np.linalg.norm(Qb, axis=1)).max() <= 1e-8
    Xo = _block64_oracle(p, Qb)
    err = np.linalg.norm(Uh - Xo, axis=1) / np.linalg.norm(Xo, axis=1)
    assert err.max() < 1e-5, err.max()


def test_nonfinite_rhs_rejected():
    p = synth.gradient_2d(n=32, nsrc=(2,), levels=3)
    Qn = p.Q.copy()
    Qn[0, 5] = np.nan
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, levels=3)
    Q = dev(Qn)
    U = torch.zeros_like(Q)
    with pytest.raises(pk.HelmError) as e:
        pk.helm_solve_block(hd, Q, U, tol=1e-7)
    assert e.value.status == pk.HELM_ERR_NONFINITE


def test_not_converged_reports_last_iterate():
    p = synth.gradient_2d(n=64, nsrc=(2,), levels=3)
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, levels=3)
    Q = dev(p.Q)
    U = torch.zeros_like(Q)
    info = pk.helm_solve_block(hd, Q, U, tol=1e-12, restart=5, max_cycles=3)
    assert info["status"] == pk.HELM_ERR_NOT_CONVERGED and not info["converged_all"]
    assert info["cycles"] == 3
    rr = pk.helm_residual(hd, Q, U)
    assert np.allclose(rr, info["relres"], rtol=1e-6)
    assert (rr < 1.0).all()  # the iterate improved on U = 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("nrhs", [6, 16, 64])
def test_fine_tile_choices_are_bitwise_identical(precision, nrhs):
    """Every tile shape of the 3D finest-level kernels (register-blocked rows,
    or the LDS-blocked 16 x 16 / 16 x 8 tiles where the block holds whole
    128 B column groups: 16 RHS in mixed, 8 in FP64; with those tiles the
    residual and the restriction run fused) computes each output from the
    same values in the same order: the cycle output must not change by a
    bit. Each tile gets a fresh handle (no buffer keeps values of another
    tile's run); inputs are dense random and sparse point sources (the
    benchmark's right-hand sides). The 47^3 grid leaves ragged x/y tiles,
    coarse tiles and z chunks."""
    p = synth.layered_3d(n=48, nsrc=(3, 2), levels=3, seed=2)
    F = dev(crand(nrhs, p.N))
    S = np.zeros((nrhs, p.N), complex)
    for c in range(nrhs):
        S[c, (37 * c + 11) % p.N] = 1e6 * (1 + 1j) / (c + 1)
        S[c, (c * 48 * 48) % p.N] = -2e6  # on the first planes and faces
    S = dev(S)
    outs = []
    for ry, zc in [(1, 16), (2, 32), (4, 64), (4, 7), (16, 16), (16, 7), (16, 64), (8, 32), (8, 5)]:
        hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, levels=3, precision=precision, coarse="lu")
        pk.helm_set_fine_tile(hd, nrhs, ry, zc)
        res = []
        for X in (F, S):
            Z = torch.empty_like(X)
            pk.helm_precond(hd, X, Z)
            res.append(host(Z))
        outs.append(res)
        del hd
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0])
        assert np.array_equal(o[1], outs[0][1])
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, levels=3, precision=precision, coarse="lu")
    ry, zc = pk.helm_fine_tile(hd, nrhs)
    assert ry in (1, 2, 4, 8, 16) and zc >= 1


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_residual_restriction_across_z_chunks(precision):
    """The fused residual + restriction marches through chunks of coarse
    planes; on 80^3 cells the coarse grid has 39 planes, more than one chunk
    with a ragged last one. The fused tile (16 x 16) and a register-blocked
    tile (residual, then restriction) must give a bitwise equal cycle."""
    p = synth.layered_3d(n=80, nsrc=(3, 2), levels=3, seed=2)
    X = dev(crand(16, p.N))
    outs = []
    for ry, zc in [(4, 16), (16, 16), (16, 64)]:
        hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, levels=3, precision=precision, coarse="lu")
        assert pk.helm_level_dims(hd, 1)[2] == 39
        pk.helm_set_fine_tile(hd, 16, ry, zc)
        Z = torch.empty_like(X)
        pk.helm_precond(hd, X, Z)
        outs.append(host(Z))
        del hd
    assert np.isfinite(outs[0]).all()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("dim,n,nrhs", [(2, 40, 1), (2, 24, 7), (3, 16, 3), (3, 33 * 2, 256)])
def test_residual_matches_oracle(dim, n, nrhs):
    """helm_residual (one pass over Q and U in the ABI layout) against the
    oracle's operator: relative residuals of random blocks agree to 1e-12
    (FP64 sums of <= 8 terms per entry, reductions of N terms); a zero
    column reports 0; the 256-column case fills every column slot of the
    partial-sum buffer."""
    p = small_problem(dim, n, 2)
    hd = pk.helm_setup(p.dim, p.n, p.h, p.m, p.gamma, p.omega, levels=2)
    g = oracle.grid(p.dim, p.n, p.h)
    Q = crand(nrhs, p.N)
    U = crand(nrhs, p.N)
    U *= 0.3 / np.abs(oracle.apply_fine(g, p.m, p.gamma, p.omega, 0.0, U[:1])).mean()
    if nrhs > 1:
        Q[1] = 0.0
    rr = pk.helm_residual(hd, dev(Q), dev(U))
    R = Q - oracle.apply_fine(g, p.m, p.gamma, p.omega, 0.0, U)
    qn = np.linalg.norm(Q, axis=1)
    ref = np.where(qn > 0, np.linalg.norm(R, axis=1) / np.where(qn > 0, qn, 1.0), 0.0)
    assert np.allclose(rr, ref, rtol=1e-12, atol=0.0), np.abs(rr - ref).max()
    if nrhs > 1:
        assert rr[1] == 0.0
