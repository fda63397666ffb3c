"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks an oracle routine against an independent construction
(scipy/numpy assembled from the textbook definitions), a closed form, an
invariant or a special case, chosen so that a dropped term, a wrong sign or
index, or a transposed operand in the oracle fails at least one of them.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import oracle
import synth

RNG = np.random.default_rng(1234)


# ---------------------------------------------------------------------------
# Independent textbook constructions (scipy.sparse), used only as references
# ---------------------------------------------------------------------------
def lap1d(n, h):
    N = n - 1
    return sp.diags([-np.ones(N - 1), 2 * np.ones(N), -np.ones(N - 1)], [-1, 0, 1]) / h ** 2


def kron_axes(mats):
    """Kronecker product for a grid whose axis 0 is fastest: mats[0] acts on axis 0."""
    out = mats[-1]
    for M in mats[-2::-1]:
        out = sp.kron(out, M)
    return out.tocsr()


def sparse_H(dim, n, h, m, gamma, omega, beta):
    mats = []
    for a in range(dim):
        ops = [sp.identity(n[b] - 1) for b in range(dim)]
        ops[a] = lap1d(n[a], h[a])
        mats.append(kron_axes(ops))
    L = sum(mats)
    return (L - sp.diags(omega ** 2 * m.ravel() * (1 - 1j * (gamma.ravel() + beta)))).tocsr()


def P1d(n):
    """1D linear interpolation: n cells -> n/2 cells (vertex-centred)."""
    Nf, Nc = n - 1, n // 2 - 1
    P = np.zeros((Nf, Nc))
    for I in range(Nc):
        i = 2 * I + 1
        P[i, I] = 1.0
        P[i - 1, I] = 0.5
        P[i + 1, I] = 0.5
    return sp.csr_matrix(P)


def sparse_P(dim, n):
    return kron_axes([P1d(n[a]) for a in range(dim)])


def stencil_to_sparse(g, st):
    """Sparse matrix of a 27-entry stencil on oracle grid g."""
    nx, ny, nz = g.nu[0], g.nu[1], g.nu[2]
    N = nx * ny * nz
    rows, cols, vals = [], [], []
    for i in range(N):
        x, y, z = i % nx, (i // nx) % ny, i // (nx * ny)
        for o in range(27):
            ox, oy, oz = o % 3 - 1, (o // 3) % 3 - 1, o // 9 - 1
            X, Y, Z = x + ox, y + oy, z + oz
            if 0 <= X < nx and 0 <= Y < ny and 0 <= Z < nz and st[i, o] != 0:
                rows.append(i)
                cols.append(X + nx * (Y + ny * Z))
                vals.append(st[i, o])
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def rand_model(dim, n):
    shape = (n - 1,) * dim
    m = 1.0 / RNG.uniform(1.5, 4.5, shape) ** 2
    gamma = RNG.uniform(0.0, 0.3, shape)
    return m, gamma


def crand(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


CASES = [(2, 8), (3, 6), (2, 12), (3, 8)]


# ---------------------------------------------------------------------------
# Operator (eq:helm / eq:LinearSystem)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,n", CASES)
@pytest.mark.parametrize("beta", [0.0, 0.2])
def test_apply_fine_matches_kronecker_assembly(dim, n, beta):
    h = tuple(1.0 / n * (1 + 0.1 * a) for a in range(dim))  # anisotropic spacing
    m, gamma = rand_model(dim, n)
    omega = 7.3
    g = oracle.grid(dim, (n,) * dim, h)
    U = crand(3, (n - 1) ** dim)
    ref = (sparse_H(dim, (n,) * dim, h, m, gamma, omega, beta) @ U.T).T
    out = oracle.apply_fine(g, m, gamma, omega, beta, U)
    assert np.allclose(out, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("dim,n", CASES)
def test_fine_stencil_equals_definition(dim, n):
    h = (1.0 / n,) * dim
    m, gamma = rand_model(dim, n)
    g = oracle.grid(dim, (n,) * dim, h)
    U = crand(2, (n - 1) ** dim)
    st = oracle.fine_stencil(g, m, gamma, 5.0, 0.2)
    a = oracle.apply_stencil(g, st, U)
    b = oracle.apply_fine(g, m, gamma, 5.0, 0.2, U)
    assert np.allclose(a, b, rtol=1e-14, atol=1e-12)


def test_operator_complex_symmetric():
    dim, n = 3, 8
    m, gamma = rand_model(dim, n)
    g = oracle.grid(dim, (n,) * dim, (1 / n,) * dim)
    x, y = crand(1, (n - 1) ** 3), crand(1, (n - 1) ** 3)
    Hx = oracle.apply_fine(g, m, gamma, 9.0, 0.0, x)
    Hy = oracle.apply_fine(g, m, gamma, 9.0, 0.0, y)
    assert abs(np.sum(y * Hx) - np.sum(x * Hy)) < 1e-10 * abs(np.sum(y * Hx))


@pytest.mark.parametrize("dim,n", [(2, 16), (3, 10)])
def test_dst_eigenpairs_constant_medium(dim, n):
    """Sine modes are eigenvectors; lambda = sum 4/h^2 sin^2(k pi / 2n) - w^2 m (1 - i g)."""
    h = 1.0 / n
    m0, g0, omega = 0.3, 0.05, 11.0
    shape = (n - 1,) * dim
    m = np.full(shape, m0)
    gamma = np.full(shape, g0)
    g = oracle.grid(dim, (n,) * dim, (h,) * dim)
    k = [3, 5, 2][:dim]
    idx = np.arange(1, n)
    mode = np.ones(())
    for a in range(dim):  # axis 0 fastest -> numpy last axis
        s = np.sin(np.pi * k[a] * idx / n)
        mode = np.multiply.outer(s, mode) if a > 0 else s
    mode = mode.reshape(1, -1).astype(complex)
    lam = sum(4 / h ** 2 * np.sin(kk * np.pi / (2 * n)) ** 2 for kk in k) - omega ** 2 * m0 * (1 - 1j * g0)
    out = oracle.apply_fine(g, m, gamma, omega, 0.0, mode)
    assert np.allclose(out, lam * mode, rtol=1e-12, atol=1e-9 * abs(lam))


# ---------------------------------------------------------------------------
# Transfers: bilinear/trilinear P and full weighting R = 2^-d P^T
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,n", [(2, 8), (2, 16), (3, 8)])
def test_prolong_restrict_match_kron(dim, n):
    g = oracle.grid(dim, (n,) * dim, (1 / n,) * dim)
    P = sparse_P(dim, (n,) * dim)
    E = crand(2, P.shape[1])
    R = crand(2, P.shape[0])
    assert np.allclose(oracle.prolong(g, E), (P @ E.T).T, atol=1e-14)
    assert np.allclose(oracle.restrict(g, R), (P.T @ R.T).T / 2 ** dim, atol=1e-14)


def test_prolong_reproduces_linear_functions_inside():
    n = 16
    g = oracle.grid(2, (n, n), (1 / n, 1 / n))
    xc = np.arange(1, n // 2) * 2.0  # coarse node positions in fine cells
    f = lambda x, z: 0.7 * x - 0.3 * z + 2.0
    E = f(xc[None, :], xc[:, None]).reshape(1, -1).astype(complex)
    U = oracle.prolong(g, E).reshape(n - 1, n - 1)
    xf = np.arange(1, n, dtype=float)
    ref = f(xf[None, :], xf[:, None])
    inner = (slice(1, -1), slice(1, -1))  # nodes whose parents are all inside
    assert np.allclose(U[inner], ref[inner], atol=1e-13)


def test_1d_transfer_identities():
    """In 1D, R P = [1, 6, 1]/8 and R A P = (1/H^2)[-1, 2, -1] (H = 2h)."""
    n = 16
    h = 1.0 / n
    P = P1d(n).toarray()
    R = P.T / 2
    RP = R @ P
    assert np.allclose(np.diag(RP), 6 / 8) and np.allclose(np.diag(RP, 1), 1 / 8)
    RAP = R @ lap1d(n, h).toarray() @ P
    H = 2 * h
    assert np.allclose(np.diag(RAP), 2 / H ** 2) and np.allclose(np.diag(RAP, 1), -1 / H ** 2)


# ---------------------------------------------------------------------------
# Galerkin coarse operators (R A P), by probing in the oracle
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,n", [(2, 16), (3, 8)])
def test_galerkin_matches_triple_product(dim, n):
    h = (1.0 / n,) * dim
    m, gamma = rand_model(dim, n)
    omega, beta = 8.0, 0.2
    g = oracle.grid(dim, (n,) * dim, h)
    M = sparse_H(dim, (n,) * dim, h, m, gamma, omega, beta)
    P = sparse_P(dim, (n,) * dim)
    Mc_ref = (P.T @ M @ P) / 2 ** dim
    stc = oracle.galerkin(g, m=m, gamma=gamma, omega=omega, beta=beta)
    gc = oracle.coarsen(g)
    assert np.allclose(stencil_to_sparse(gc, stc).toarray(), Mc_ref.toarray(), atol=1e-12 * abs(Mc_ref).max())
    # second level from the stencil form
    P2 = sparse_P(dim, (n // 2,) * dim)
    Mcc_ref = (P2.T @ Mc_ref @ P2) / 2 ** dim
    stcc = oracle.galerkin(gc, st=stc)
    gcc = oracle.coarsen(gc)
    assert np.allclose(stencil_to_sparse(gcc, stcc).toarray(), Mcc_ref.toarray(), atol=1e-12 * abs(Mcc_ref).max())


def test_galerkin_closed_form_constant_coefficients():
    """M_c = (1/H^2) sum_d K_d (x) S (x) S - w^2 m (1 - i(g+b)) S (x) S (x) S,
    K = [-1, 2, -1], S = [1, 6, 1]/8, at every coarse node (Dirichlet truncated)."""
    n, dim = 16, 3
    h = 1.0 / n
    m0, g0, beta, omega = 0.25, 0.1, 0.2, 13.0
    shape = (n - 1,) * dim
    g = oracle.grid(dim, (n,) * dim, (h,) * dim)
    stc = oracle.galerkin(g, m=np.full(shape, m0), gamma=np.full(shape, g0), omega=omega, beta=beta)
    H = 2 * h
    K = {-1: -1.0, 0: 2.0, 1: -1.0}
    S = {-1: 1 / 8, 0: 6 / 8, 1: 1 / 8}
    mass = -omega ** 2 * m0 * (1 - 1j * (g0 + beta))
    ref = np.zeros(27, complex)
    for o in range(27):
        ox, oy, oz = o % 3 - 1, (o // 3) % 3 - 1, o // 9 - 1
        lap = (K[ox] * S[oy] * S[oz] + S[ox] * K[oy] * S[oz] + S[ox] * S[oy] * K[oz]) / H ** 2
        ref[o] = lap + mass * S[ox] * S[oy] * S[oz]
    gc = oracle.coarsen(g)
    nc = gc.nu[0]
    # interior node: every entry; boundary nodes: the entries that stay inside
    for (x, y, z) in [(3, 3, 3), (0, 0, 0), (nc - 1, 2, 0)]:
        i = x + nc * (y + nc * z)
        for o in range(27):
            ox, oy, oz = o % 3 - 1, (o // 3) % 3 - 1, o // 9 - 1
            inside = all(0 <= c + d < nc for c, d in ((x, ox), (y, oy), (z, oz)))
            assert abs(stc[i, o] - (ref[o] if inside else 0)) < 1e-10 * abs(ref).max()


def test_galerkin_complex_symmetric():
    dim, n = 3, 8
    m, gamma = rand_model(dim, n)
    g = oracle.grid(dim, (n,) * dim, (1 / n,) * dim)
    stc = oracle.galerkin(g, m=m, gamma=gamma, omega=6.0, beta=0.2)
    A = stencil_to_sparse(oracle.coarsen(g), stc).toarray()
    assert np.allclose(A, A.T, atol=1e-12 * abs(A).max())


# ---------------------------------------------------------------------------
# Damped Jacobi (section 5.3)
# ---------------------------------------------------------------------------
def test_jacobi_sine_mode_amplification():
    n, dim = 16, 2
    h = 1.0 / n
    m0, g0, beta, omega, w = 0.3, 0.02, 0.2, 12.0, 0.8
    g = oracle.grid(dim, (n,) * dim, (h,) * dim)
    shape = (n - 1,) * dim
    st = oracle.fine_stencil(g, np.full(shape, m0), np.full(shape, g0), omega, beta)
    idx = np.arange(1, n)
    k = (4, 7)
    mode = np.outer(np.sin(np.pi * k[1] * idx / n), np.sin(np.pi * k[0] * idx / n)).reshape(1, -1).astype(complex)
    lam = sum(4 / h ** 2 * np.sin(kk * np.pi / (2 * n)) ** 2 for kk in k) - omega ** 2 * m0 * (1 - 1j * (g0 + beta))
    D = 4 / h ** 2 - omega ** 2 * m0 * (1 - 1j * (g0 + beta))
    out = oracle.jacobi(g, st, w, 1, np.zeros_like(mode), U0=mode)
    assert np.allclose(out, (1 - w * lam / D) * mode, atol=1e-12)


# ---------------------------------------------------------------------------
# Dense helpers and the coarsest LU
# ---------------------------------------------------------------------------
def test_householder_qr():
    A = crand(5, 200)  # [p][N]
    Q, R = oracle.householder_qr(A)
    Qm = Q.T
    assert np.allclose(Qm.conj().T @ Qm, np.eye(5), atol=1e-13)
    assert np.allclose(Qm @ R, A.T, atol=1e-12)
    assert np.allclose(np.tril(R, -1), 0)


def test_householder_qr_rank_revealing():
    """Rank-revealing QR (the block method's deflation of dependent
    directions): duplicate and combined columns are dropped, Q spans the
    columns' space with orthonormal columns up to the rank and zero columns
    past it, R has zero rows past the rank, and Q R reproduces the input."""
    a = crand(3, 300)
    A = np.stack([a[0], a[1], a[0], a[0] + 2 * a[1], a[2]])  # rank 3
    Q, R, r = oracle.householder_qr_rr(A)
    assert r == 3 == np.linalg.matrix_rank(A.T)
    Qm = Q.T
    assert np.allclose(Qm.conj().T @ Qm, np.diag([1, 1, 1, 0, 0]), atol=1e-13)
    assert np.abs(Qm[:, 3:]).max() == 0.0 and np.abs(R[3:]).max() == 0.0
    assert np.allclose(Qm @ R, A.T, atol=1e-12 * np.abs(A).max())
    # duplicate columns keep identical coefficients
    assert np.allclose(R[:, 0], R[:, 2], atol=1e-13 * np.abs(R).max())
    # a dependence weaker than the tolerance is kept as a direction
    B = A.copy()
    B[2] = a[0] + 1e-9 * crand(1, 300)[0]
    Qb, Rb, rb = oracle.householder_qr_rr(B)
    assert rb == 4
    assert np.allclose(Qb.T @ Rb, B.T, atol=1e-12 * np.abs(B).max())
    # full rank: the same factor as the unpivoted QR up to column phases
    C = crand(4, 200)
    Qc, Rc, rc = oracle.householder_qr_rr(C)
    Q0, R0 = oracle.householder_qr(C)
    assert rc == 4
    assert np.allclose(Qc.T @ Rc, C.T, atol=1e-12)
    assert np.allclose(np.abs(Qc.conj() @ Qc.T), np.eye(4), atol=1e-13)
    # the same column space as the unpivoted Q
    assert np.allclose(Q0.T @ (Q0.conj() @ Qc.T), Qc.T, atol=1e-12)


def test_lstsq_matches_numpy():
    A = crand(14, 9)
    B = crand(14, 3)
    Y, res = oracle.lstsq(A, B)
    Yr = np.linalg.lstsq(A, B, rcond=None)[0]
    assert np.allclose(Y, Yr, atol=1e-12)
    assert np.allclose(res, np.linalg.norm(B - A @ Yr, axis=0), atol=1e-12)


@pytest.mark.parametrize("dim,n,levels", [(2, 16, 2), (3, 8, 2), (2, 32, 3)])
def test_coarsest_band_lu_equals_dense_solve(dim, n, levels):
    m, gamma = rand_model(dim, n)
    g = oracle.grid(dim, (n,) * dim, (1 / n,) * dim)
    H = oracle.Hierarchy(g, m, gamma, 9.0, 0.2, levels)
    gc = H.level_grid(levels - 1)
    A = stencil_to_sparse(gc, H.stencil(levels - 1)).toarray()
    F = crand(3, A.shape[0])
    assert np.allclose(H.coarse_solve(F), np.linalg.solve(A, F.T).T, atol=1e-11 * np.abs(F).max())


# ---------------------------------------------------------------------------
# V-cycle: the two-grid cycle applied recursively, as a fixed linear map
# ---------------------------------------------------------------------------
def dense_vcycle(Ms, Ps, f, l, w, nu, coarse, dim, wcycle=False):
    """The two-grid cycle with dense matrices, recursively. W-cycle: a coarse
    problem other than the coarsest gets a second cycle on the residual of
    the first, e += B(r_c - M_c e)."""
    if l == len(Ms) - 1:
        return coarse(Ms[l], f)
    M = Ms[l]
    Dinv = 1.0 / np.diag(M)
    u = np.zeros_like(f)
    for _ in range(nu):
        u = u + w * Dinv * (f - M @ u)
    rc = Ps[l].T @ (f - M @ u) / 2 ** dim
    e = dense_vcycle(Ms, Ps, rc, l + 1, w, nu, coarse, dim, wcycle)
    if wcycle and l + 1 < len(Ms) - 1:
        e = e + dense_vcycle(Ms, Ps, rc - Ms[l + 1] @ e, l + 1, w, nu, coarse, dim, wcycle)
    u = u + Ps[l] @ e
    for _ in range(nu):
        u = u + w * Dinv * (f - M @ u)
    return u


def dense_hierarchy(dim, n, m, gamma, omega, beta, levels):
    h = (1.0 / n,) * dim
    Ms = [sparse_H(dim, (n,) * dim, h, m, gamma, omega, beta).toarray()]
    Ps = []
    nn = n
    for _ in range(levels - 1):
        P = sparse_P(dim, (nn,) * dim).toarray()
        Ps.append(P)
        Ms.append(P.T @ Ms[-1] @ P / 2 ** dim)
        nn //= 2
    return Ms, Ps


def np_gmres_fixed(A, b, k):
    """k steps of GMRES from zero: minimiser of ||b - A x|| over K_k(A, b)."""
    beta = np.linalg.norm(b)
    V = np.zeros((len(b), k + 1), complex)
    Hm = np.zeros((k + 1, k), complex)
    V[:, 0] = b / beta
    for j in range(k):
        w = A @ V[:, j]
        for i in range(j + 1):
            Hm[i, j] = np.vdot(V[:, i], w)
            w = w - Hm[i, j] * V[:, i]
        Hm[j + 1, j] = np.linalg.norm(w)
        V[:, j + 1] = w / Hm[j + 1, j]
    e1 = np.zeros(k + 1, complex)
    e1[0] = beta
    y = np.linalg.lstsq(Hm, e1, rcond=None)[0]
    return V[:, :k] @ y


@pytest.mark.parametrize("dim,n,levels", [(2, 16, 3), (3, 8, 2), (3, 16, 3)])
def test_vcycle_equals_dense_composition(dim, n, levels):
    m, gamma = rand_model(dim, n)
    omega, beta = 10.0, 0.2
    Ms, Ps = dense_hierarchy(dim, n, m, gamma, omega, beta, levels)
    g = oracle.grid(dim, (n,) * dim, (1 / n,) * dim)
    H = oracle.Hierarchy(g, m, gamma, omega, beta, levels)
    F = crand(2, Ms[0].shape[0])
    out = H.vcycle(F)
    for s in range(2):
        ref = dense_vcycle(Ms, Ps, F[s], 0, 0.8, 2, lambda A, b: np.linalg.solve(A, b), dim)
        assert np.allclose(out[s], ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("dim,n,levels", [(2, 32, 4), (3, 16, 3)])
def test_wcycle_equals_dense_composition(dim, n, levels):
    m, gamma = rand_model(dim, n)
    omega, beta = 10.0, 0.2
    Ms, Ps = dense_hierarchy(dim, n, m, gamma, omega, beta, levels)
    g = oracle.grid(dim, (n,) * dim, (1 / n,) * dim)
    H = oracle.Hierarchy(g, m, gamma, omega, beta, levels, cycle="W")
    F = crand(2, Ms[0].shape[0])
    out = H.vcycle(F)
    solve = lambda A, b: np.linalg.solve(A, b)
    for s in range(2):
        ref = dense_vcycle(Ms, Ps, F[s], 0, 0.8, 2, solve, dim, wcycle=True)
        assert np.allclose(out[s], ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
        v = dense_vcycle(Ms, Ps, F[s], 0, 0.8, 2, solve, dim)
        assert np.linalg.norm(ref - v) > 1e-3 * np.linalg.norm(v)  # the W-cycle is another map


def dense_kcycle(Ms, Ps, f, l, w, nu, coarse, dim):
    """The cycle with the K-cycle coarse correction, densely: a coarse level
    other than the coarsest is solved by the minimal residual over the
    flexible Krylov space of two steps, span{z1, z2} with z1 = B v1,
    v1 = r / ||r||, z2 = B v2 and v2 the part of M z1 orthogonal to v1
    (normalised), B the level's own K-cycle: e = Z argmin ||r - M Z y||."""
    if l == len(Ms) - 1:
        return coarse(Ms[l], f)
    M = Ms[l]
    Dinv = 1.0 / np.diag(M)
    u = np.zeros_like(f)
    for _ in range(nu):
        u = u + w * Dinv * (f - M @ u)
    rc = Ps[l].T @ (f - M @ u) / 2 ** dim
    if l + 1 < len(Ms) - 1:
        Mc = Ms[l + 1]
        B = lambda v: dense_kcycle(Ms, Ps, v, l + 1, w, nu, coarse, dim)
        v1 = rc / np.linalg.norm(rc)
        z1 = B(v1)
        t = Mc @ z1
        t = t - np.vdot(v1, t) * v1
        z2 = B(t / np.linalg.norm(t))
        Z = np.stack([z1, z2], axis=1)
        y = np.linalg.lstsq(Mc @ Z, rc, rcond=None)[0]
        e = Z @ y
    else:
        e = dense_kcycle(Ms, Ps, rc, l + 1, w, nu, coarse, dim)
    u = u + Ps[l] @ e
    for _ in range(nu):
        u = u + w * Dinv * (f - M @ u)
    return u


@pytest.mark.parametrize("dim,n,levels", [(2, 32, 3), (2, 32, 4), (3, 16, 3)])
def test_kcycle_equals_dense_minimal_residual(dim, n, levels):
    """The K-cycle (two flexible GMRES steps on every coarse level but the
    coarsest) equals its definition as a minimal residual over the flexible
    Krylov space, and differs from the V-cycle."""
    m, gamma = rand_model(dim, n)
    omega, beta = 10.0, 0.2
    Ms, Ps = dense_hierarchy(dim, n, m, gamma, omega, beta, levels)
    g = oracle.grid(dim, (n,) * dim, (1 / n,) * dim)
    H = oracle.Hierarchy(g, m, gamma, omega, beta, levels, cycle="K")
    F = crand(2, Ms[0].shape[0])
    out = H.vcycle(F)
    solve = lambda A, b: np.linalg.solve(A, b)
    for s in range(2):
        ref = dense_kcycle(Ms, Ps, F[s], 0, 0.8, 2, solve, dim)
        assert np.allclose(out[s], ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())
        v = dense_vcycle(Ms, Ps, F[s], 0, 0.8, 2, solve, dim)
        assert np.linalg.norm(ref - v) > 1e-3 * np.linalg.norm(v)


def jacobi_from_zero(A, b, w, sweeps):
    u = np.zeros_like(b)
    Dinv = 1.0 / np.diag(A)
    for _ in range(sweeps):
        u = u + w * Dinv * (b - A @ u)
    return u


@pytest.mark.parametrize("dim,n,levels", [(2, 16, 3), (3, 16, 3)])
def test_vcycle_with_relaxed_coarsest_equals_dense(dim, n, levels):
    """Relaxation-only coarsest level: nu_pre + nu_post damped Jacobi sweeps
    from zero with that level's weight (here 2 + 2 at 0.8)."""
    m, gamma = rand_model(dim, n)
    omega, beta = 10.0, 0.2
    Ms, Ps = dense_hierarchy(dim, n, m, gamma, omega, beta, levels)
    g = oracle.grid(dim, (n,) * dim, (1 / n,) * dim)
    H = oracle.Hierarchy(g, m, gamma, omega, beta, levels, coarse="none")
    F = crand(2, Ms[0].shape[0])
    out = H.vcycle(F)
    for s in range(2):
        ref = dense_vcycle(Ms, Ps, F[s], 0, 0.8, 2, lambda A, b: jacobi_from_zero(A, b, 0.8, 4), dim)
        assert np.allclose(out[s], ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
    C = Ms[-1]
    Fc = crand(3, C.shape[0])
    assert np.allclose(H.coarse_solve(Fc), np.array([jacobi_from_zero(C, f, 0.8, 4) for f in Fc]),
                       atol=1e-12 * np.abs(Fc).max())


@pytest.mark.parametrize("k", [3, 8])
def test_vcycle_with_gmres_coarsest_equals_dense(k):
    dim, n, levels = 2, 32, 3
    m, gamma = rand_model(dim, n)
    omega, beta = 20.0, 0.2
    Ms, Ps = dense_hierarchy(dim, n, m, gamma, omega, beta, levels)
    g = oracle.grid(dim, (n,) * dim, (1 / n,) * dim)
    H = oracle.Hierarchy(g, m, gamma, omega, beta, levels, coarse="gmres", coarse_iters=k)
    F = crand(2, Ms[0].shape[0])
    out = H.vcycle(F)
    for s in range(2):
        ref = dense_vcycle(Ms, Ps, F[s], 0, 0.8, 2, lambda A, b: np_gmres_fixed(A, b, k), dim)
        assert np.allclose(out[s], ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_coarse_gmres_restarts_equal_krylov_minimisers():
    """Restarted GMRES(k) on the coarsest grid: every restart adds the
    minimiser of ||r - A d|| over the Krylov space K_k(A, r) of the current
    residual r. The reference builds the explicit Krylov matrix [r, Ar, ...]
    and solves that least-squares problem directly (no Arnoldi); the residual
    never grows from one restart to the next, and one restart is the plain
    fixed-step solve."""
    dim, n, levels, k = 2, 16, 2, 3
    m, gamma = rand_model(dim, n)
    omega, beta = 12.0, 0.2
    Ms, Ps = dense_hierarchy(dim, n, m, gamma, omega, beta, levels)
    A = Ms[-1]
    g = oracle.grid(dim, (n,) * dim, (1 / n,) * dim)
    F = crand(2, A.shape[0])
    res = []
    for R in (1, 2, 3):
        H = oracle.Hierarchy(g, m, gamma, omega, beta, levels, coarse="gmres", coarse_iters=k, coarse_restarts=R)
        out = H.coarse_solve(F)
        for s in range(2):
            x = np.zeros(A.shape[0], complex)
            for _ in range(R):
                r = F[s] - A @ x
                K = np.empty((len(r), k), complex)
                K[:, 0] = r / np.linalg.norm(r)
                for j in range(1, k):
                    K[:, j] = A @ K[:, j - 1]
                    K[:, j] /= np.linalg.norm(K[:, j])
                y = np.linalg.lstsq(A @ K, r, rcond=None)[0]
                x = x + K @ y
            assert np.allclose(out[s], x, rtol=1e-9, atol=1e-9 * np.abs(x).max())
        res.append(np.linalg.norm(F - out @ A.T, axis=1))
    assert np.all(res[1] <= res[0] * (1 + 1e-12)) and np.all(res[2] <= res[1] * (1 + 1e-12))
    H1 = oracle.Hierarchy(g, m, gamma, omega, beta, levels, coarse="gmres", coarse_iters=k)
    assert np.array_equal(H1.coarse_solve(F), oracle.Hierarchy(g, m, gamma, omega, beta, levels, coarse="gmres",
                                                               coarse_iters=k, coarse_restarts=1).coarse_solve(F))


def test_vcycle_poisson_contraction():
    """omega = 0: V(2,2) with damped Jacobi is a convergent solver for the
    Laplacian; per-cycle error reduction stays well below the 2D smoothing
    bound (0.6^4 = 0.13 for weight 0.8) times a small constant."""
    dim, n = 2, 64
    shape = (n - 1,) * dim
    g = oracle.grid(dim, (n,) * dim, (1 / n,) * dim)
    m, gamma = np.ones(shape), np.zeros(shape)
    H = oracle.Hierarchy(g, m, gamma, 0.0, 0.0, 4)
    x_true = crand(1, (n - 1) ** 2)
    f = oracle.apply_fine(g, m, gamma, 0.0, 0.0, x_true)
    x = np.zeros_like(x_true)
    errs = []
    for _ in range(6):
        x = x + H.vcycle(f - oracle.apply_fine(g, m, gamma, 0.0, 0.0, x))
        errs.append(np.linalg.norm(x - x_true))
    rates = np.array(errs[1:]) / np.array(errs[:-1])
    assert rates.max() < 0.2


# ---------------------------------------------------------------------------
# Block FGMRES (section 5.3)
# ---------------------------------------------------------------------------
def test_fgmres_identity_prec_equals_scipy_gmres():
    dim, n = 2, 16
    m, gamma = rand_model(dim, n)
    omega = 6.0
    g = oracle.grid(dim, (n,) * dim, (1 / n,) * dim)
    A = sparse_H(dim, (n,) * dim, (1 / n,) * dim, m, gamma, omega, 0.0)
    H = oracle.Hierarchy(g, m, gamma, omega, 0.2, 2)
    q = crand(1, A.shape[0])
    restart, cycles = 6, 4
    X, it, rr, conv = H.fgmres(q, tol=1e-30, restart=restart, maxit=restart * cycles, prec=False)
    assert it == restart * cycles
    xs, _ = spl.gmres(A, q[0], x0=np.zeros_like(q[0]), rtol=1e-30, atol=0.0, restart=restart, maxiter=cycles)
    assert np.allclose(X[0], xs, rtol=1e-8, atol=1e-8 * np.abs(xs).max())


def test_block_fgmres_saturates_to_exact_in_one_cycle():
    dim, n = 2, 8  # N = 49
    m, gamma = rand_model(dim, n)
    g = oracle.grid(dim, (n,) * dim, (1 / n,) * dim)
    A = sparse_H(dim, (n,) * dim, (1 / n,) * dim, m, gamma, 9.0, 0.0).toarray()
    H = oracle.Hierarchy(g, m, gamma, 9.0, 0.2, 2)
    Q = crand(7, 49)
    X, it, rr, conv = H.fgmres(Q, tol=1e-13, restart=7, maxit=7, prec=False)
    assert np.allclose(X, np.linalg.solve(A, Q.T).T, atol=1e-10 * np.abs(X).max())


@pytest.mark.parametrize("p", [1, 3])
def test_fgmres_manufactured_solution(p):
    dim, n = 3, 16
    m, gamma = rand_model(dim, n)
    omega = 25.0
    g = oracle.grid(dim, (n,) * dim, (1 / n,) * dim)
    H = oracle.Hierarchy(g, m, gamma, omega, 0.2, 3)
    Ustar = crand(p, (n - 1) ** 3)
    Q = oracle.apply_fine(g, m, gamma, omega, 0.0, Ustar)
    X, it, rr, conv = H.fgmres(Q, tol=1e-11, restart=5, maxit=300)
    assert conv and rr.max() <= 1e-11
    assert np.linalg.norm(X - Ustar) / np.linalg.norm(Ustar) < 1e-8


def test_fgmres_converged_columns_meet_tolerance_and_dense_solution():
    p = synth.gradient_2d(n=32, nsrc=(3,), levels=3)
    g = oracle.grid(p.dim, p.n, p.h)
    H = oracle.setup_problem(p)
    X, it, rr, conv = H.fgmres(p.Q, tol=1e-8, restart=10, maxit=500)
    assert conv and rr.max() <= 1e-8
    A = sparse_H(2, p.n, p.h, p.m, p.gamma, p.omega, 0.0)
    Xd = spl.splu(A.tocsc()).solve(p.Q.T).T
    assert np.linalg.norm(X - Xd) / np.linalg.norm(Xd) < 1e-6


@pytest.mark.parametrize("restart", [5, 12])
def test_fgmres_duplicate_and_dependent_sources(restart):
    """A block with a duplicate source and a combination of two sources
    (rank 2 of 4): the rank-revealing QR drops the dependent directions,
    the duplicate's solution equals the first source's, the combination's
    equals the same combination of solutions, and every column meets the
    tolerance against the sparse direct solve, as the single sources do
    when solved alone."""
    p = synth.gradient_2d(n=32, nsrc=(2,), levels=3)
    H = oracle.setup_problem(p)
    q0, q1 = p.Q[0], p.Q[1]
    Q = np.stack([q0, q1, q0, q0 + 2 * q1])
    X, it, rr, conv = H.fgmres(Q, tol=1e-9, restart=restart, maxit=300)
    assert conv and rr.max() <= 1e-9 and np.isfinite(X).all()
    scale = np.abs(X).max()
    assert np.allclose(X[2], X[0], atol=1e-10 * scale)
    assert np.allclose(X[3], X[0] + 2 * X[1], atol=1e-7 * scale)
    A = sparse_H(2, p.n, p.h, p.m, p.gamma, p.omega, 0.0)
    Xd = spl.splu(A.tocsc()).solve(Q.T).T
    assert (np.linalg.norm(X - Xd, axis=1) / np.linalg.norm(Xd, axis=1)).max() < 1e-6
    Xs, _, rs, cs = H.fgmres(p.Q, tol=1e-9, restart=restart, maxit=300)
    assert cs
    assert np.linalg.norm(X[:2] - Xs) / np.linalg.norm(Xs) < 1e-6
    # the duplicate block takes no more cycles than the independent pair
    itp = H.fgmres(p.Q, tol=1e-9, restart=restart, maxit=300)[1]
    assert it <= itp + restart


def test_fgmres_warm_start_is_a_shifted_cold_solve():
    """FGMRES sees the initial guess only through its residual: a warm start
    at X0 gives X0 + (the cold solve of H D = Q - H X0), iterate for
    iterate; and a warm start at the exact solution takes no cycle."""
    p = synth.gradient_2d(n=32, nsrc=(2,), levels=3)
    H = oracle.setup_problem(p)
    g = oracle.grid(p.dim, p.n, p.h)
    X0 = crand(2, p.N) * 1e-4
    R0 = p.Q - oracle.apply_fine(g, p.m, p.gamma, p.omega, 0.0, X0)
    Xw, itw, _, _ = H.fgmres(p.Q, tol=1e-30, restart=5, maxit=12, X0=X0)
    D, itc, _, _ = H.fgmres(R0, tol=1e-30, restart=5, maxit=12)
    assert itw == itc == 12
    assert np.allclose(Xw, X0 + D, rtol=1e-10, atol=1e-10 * np.abs(Xw).max())
    A = sparse_H(2, p.n, p.h, p.m, p.gamma, p.omega, 0.0)
    Xs = spl.splu(A.tocsc()).solve(p.Q.T).T
    X, it, rr, conv = H.fgmres(p.Q, tol=1e-8, restart=5, maxit=50, X0=Xs)
    assert conv and it == 0 and np.array_equal(X, Xs)


def test_residual_estimates_track_true_residual():
    """Flexible Arnoldi identity: the LS residual is the true residual."""
    p = synth.gradient_2d(n=32, nsrc=(2,), levels=3)
    H = oracle.setup_problem(p)
    X, it, rr, conv, hist = H.fgmres(p.Q, tol=1e-9, restart=50, maxit=50, hist=True)
    g = oracle.grid(p.dim, p.n, p.h)
    true = np.linalg.norm(p.Q - oracle.apply_fine(g, p.m, p.gamma, p.omega, 0.0, X), axis=1) / np.linalg.norm(p.Q, axis=1)
    assert abs(hist[-1] - true.max()) < 1e-6 * max(true.max(), 1e-12) + 1e-12


# ---------------------------------------------------------------------------
# Physics: constant medium against the free-space Green's function
# ---------------------------------------------------------------------------
@pytest.mark.slow
def test_green_function_2d_constant_medium():
    """H u = h^-2 e_s in a constant medium with an absorbing layer on every
    face approximates the decaying free-space Green's function of -Lap - k^2,
    -(i/4) H0^(2)(k r), away from the source and the layer (O((kh)^2) phase
    error at 20 points per wavelength)."""
    from scipy.special import hankel2
    n, width = 256, 64
    h = 1.0 / n
    ppw = 24.0
    v = 2.0
    omega = synth.omega_for_ppw(v, ppw, h)
    k = omega / v
    shape = (n - 1, n - 1)
    m = np.full(shape, 1 / v ** 2)
    gamma = synth.layer_gamma(2, n, width, gmax=1.0, top=True)  # strongly absorbing
    src = (n // 2 - 1, n // 2 - 1)
    Q = synth.point_rhs(2, n, h, [src])
    g = oracle.grid(2, (n, n), (h, h))
    H = oracle.Hierarchy(g, m, gamma, omega, 0.2, 3)
    X, it, rr, conv = H.fgmres(Q, tol=1e-8, restart=20, maxit=1000)
    assert conv
    U = X.reshape(shape)
    zz, xx = np.meshgrid(np.arange(1, n) * h, np.arange(1, n) * h, indexing="ij")
    r = np.hypot(zz - (src[0] + 1) * h, xx - (src[1] + 1) * h)
    lam = 2 * np.pi / k
    ring = (r > 0.5 * lam) & (r < 2.0 * lam)
    G = -0.25j * hankel2(0, k * r[ring])
    err = np.linalg.norm(U[ring] - G) / np.linalg.norm(G)
    assert err < 0.05


@pytest.mark.slow
def test_green_function_3d_constant_medium():
    """The 3D counterpart: H u = h^-3 e_s in a constant medium with an
    absorbing layer on every face approximates exp(-i k r) / (4 pi r), the
    outgoing free-space Green's function of -Lap - k^2 for this sign
    convention, between 0.5 and 1.5 wavelengths from the source (16 points
    per wavelength: about 4.6% from the 7-point stencil's dispersion and the
    layer). A source scaled by h^-2, a conjugated phase or a growing
    damping term each miss by far more."""
    n, width = 96, 20
    h = 1.0 / n
    v = 2.0
    omega = synth.omega_for_ppw(v, 16.0, h)
    k = omega / v
    shape = (n - 1,) * 3
    m = np.full(shape, 1 / v ** 2)
    gamma = synth.layer_gamma(3, n, width, gmax=1.0, top=True)
    src = (n // 2 - 1,) * 3
    Q = synth.point_rhs(3, n, h, [src])
    g = oracle.grid(3, (n,) * 3, (h,) * 3)
    H = oracle.Hierarchy(g, m, gamma, omega, 0.2, 3)
    X, it, rr, conv = H.fgmres(Q, tol=1e-7, restart=20, maxit=200)
    assert conv
    U = X.reshape(shape)
    ax = np.arange(1, n) * h
    zz, yy, xx = np.meshgrid(ax, ax, ax, indexing="ij")
    c = (src[0] + 1) * h
    r = np.sqrt((zz - c) ** 2 + (yy - c) ** 2 + (xx - c) ** 2)
    lam = 2 * np.pi / k
    ring = (r > 0.5 * lam) & (r < 1.5 * lam)
    G = np.exp(-1j * k * r[ring]) / (4 * np.pi * r[ring])
    err = np.linalg.norm(U[ring] - G) / np.linalg.norm(G)
    assert err < 0.06
