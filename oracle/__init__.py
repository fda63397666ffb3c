"""Python view of the plain FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU
baseline use this package. The solver library never imports, links or
calls it, and it shares no code with the HIP path.

Every function takes and returns numpy arrays in the oracle's layout:
complex128 blocks ``[nrhs][N]`` with axis 0 of the grid fastest, and
27-entry stencils ``[N][27]`` (entry ``(ox+1) + 3(oy+1) + 9(oz+1)``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libhelm_oracle.so")
_lib = None


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("nu", C.c_int * 3), ("h", C.c_double * 3)]


def grid(dim: int, n, h) -> Grid:
    """Grid of ``n`` cells per axis (solver order, axis 0 fastest)."""
    g = Grid()
    g.dim = dim
    for a in range(3):
        g.nu[a] = (n[a] - 1) if a < dim else 1
        g.h[a] = h[a] if a < dim else 1.0
    return g


def npts(g: Grid) -> int:
    return g.nu[0] * g.nu[1] * g.nu[2]


def coarsen(g: Grid) -> Grid:
    c = Grid()
    lib().og_coarsen(C.byref(g), C.byref(c))
    return c


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIBPATH)
        P = C.c_void_p
        G = C.POINTER(Grid)
        L.og_npts.restype = C.c_int64
        L.og_npts.argtypes = [G]
        L.og_coarsen.argtypes = [G, G]
        L.orc_apply_fine.argtypes = [G, P, P, C.c_double, C.c_double, C.c_int, P, P]
        L.orc_fine_stencil.argtypes = [G, P, P, C.c_double, C.c_double, P]
        L.orc_apply_stencil.argtypes = [G, P, C.c_int, P, P]
        L.orc_prolong.argtypes = [G, C.c_int, P, P]
        L.orc_restrict.argtypes = [G, C.c_int, P, P]
        L.orc_galerkin.argtypes = [G, P, P, P, C.c_double, C.c_double, P]
        L.orc_jacobi.argtypes = [G, P, C.c_double, C.c_int, C.c_int, P, P]
        L.orc_setup.restype = P
        L.orc_setup.argtypes = [G, P, P, C.c_double, C.c_double, C.c_int, P, P, P, C.c_int, C.c_int]
        L.orc_free.argtypes = [P]
        L.orc_levels.argtypes = [P]
        L.orc_level_grid.argtypes = [P, C.c_int, G]
        L.orc_level_stencil.argtypes = [P, C.c_int, P]
        L.orc_vcycle.argtypes = [P, C.c_int, P, P]
        L.orc_coarse_solve.argtypes = [P, C.c_int, P, P]
        L.orc_set_coarse_restarts.argtypes = [P, C.c_int]
        L.orc_set_cycle_w.argtypes = [P, C.c_int]
        L.orc_set_cycle_k.argtypes = [P, C.c_int]
        L.orc_block_fgmres.argtypes = [P, C.c_int, C.c_int, P, P, C.c_int, C.c_double,
                                       C.c_int, C.c_int, C.POINTER(C.c_int), P, P]
        L.orc_householder_qr.argtypes = [C.c_int64, C.c_int, P, P]
        L.orc_householder_qr_rr.argtypes = [C.c_int64, C.c_int, P, P, C.c_double]
        L.orc_householder_qr_rr.restype = C.c_int
        L.orc_lstsq.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, P]
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64).ravel()


def num_threads() -> int:
    return lib().orc_num_threads()


def apply_fine(g, m, gamma, omega, beta, U):
    """(-Lap_h - omega^2 m (1 - i(gamma+beta))) U for a block [nrhs][N]."""
    U = _c(U).reshape(-1, npts(g))
    out = np.empty_like(U)
    m, gamma = _d(m), _d(gamma)
    lib().orc_apply_fine(C.byref(g), _p(m), _p(gamma), omega, beta, U.shape[0], _p(U), _p(out))
    return out


def fine_stencil(g, m, gamma, omega, beta):
    st = np.empty((npts(g), 27), np.complex128)
    m, gamma = _d(m), _d(gamma)
    lib().orc_fine_stencil(C.byref(g), _p(m), _p(gamma), omega, beta, _p(st))
    return st


def apply_stencil(g, st, U):
    U = _c(U).reshape(-1, npts(g))
    st = _c(st)
    out = np.empty_like(U)
    lib().orc_apply_stencil(C.byref(g), _p(st), U.shape[0], _p(U), _p(out))
    return out


def prolong(g, E):
    c = coarsen(g)
    E = _c(E).reshape(-1, npts(c))
    out = np.empty((E.shape[0], npts(g)), np.complex128)
    lib().orc_prolong(C.byref(g), E.shape[0], _p(E), _p(out))
    return out


def restrict(g, R):
    c = coarsen(g)
    R = _c(R).reshape(-1, npts(g))
    out = np.empty((R.shape[0], npts(c)), np.complex128)
    lib().orc_restrict(C.byref(g), R.shape[0], _p(R), _p(out))
    return out


def galerkin(g, st=None, m=None, gamma=None, omega=0.0, beta=0.0):
    c = coarsen(g)
    out = np.empty((npts(c), 27), np.complex128)
    if st is None:
        m, gamma = _d(m), _d(gamma)
        lib().orc_galerkin(C.byref(g), None, _p(m), _p(gamma), omega, beta, _p(out))
    else:
        st = _c(st)
        lib().orc_galerkin(C.byref(g), _p(st), None, None, 0.0, 0.0, _p(out))
    return out


def jacobi(g, st, w, nsweep, F, U0=None):
    F = _c(F).reshape(-1, npts(g))
    U = np.zeros_like(F) if U0 is None else _c(U0).reshape(F.shape).copy()
    st = _c(st)
    lib().orc_jacobi(C.byref(g), _p(st), w, nsweep, F.shape[0], _p(F), _p(U))
    return U


def householder_qr(A):
    """A: [p][N] (columns contiguous). Returns (Q [p][N], R column-major p x p)."""
    A = _c(A).copy()
    p, N = A.shape
    R = np.empty((p, p), np.complex128)
    lib().orc_householder_qr(N, p, _p(A), _p(R))
    return A, R.T.copy()  # R returned as a numpy matrix (row, col)


def householder_qr_rr(A, tol=1e-13):
    """Rank-revealing QR of A [p][N] (columns contiguous): (Q [p][N] with zero
    columns past the rank, R (numpy p x p, original column order), rank)."""
    A = _c(A).copy()
    p, N = A.shape
    R = np.empty((p, p), np.complex128)
    r = lib().orc_householder_qr_rr(N, p, _p(A), _p(R), float(tol))
    return A, R.T.copy(), int(r)


def lstsq(A, B):
    """min ||B - A Y||_F; A (m x n), B (m x k) numpy matrices."""
    A = np.asfortranarray(A, dtype=np.complex128)
    B = np.asfortranarray(B, dtype=np.complex128)
    mr, nc = A.shape
    k = B.shape[1]
    Y = np.empty((k, nc), np.complex128)
    res = np.empty(k)
    Af = np.ascontiguousarray(A.T)
    Bf = np.ascontiguousarray(B.T)
    lib().orc_lstsq(mr, nc, k, _p(Af), _p(Bf), _p(Y), _p(res))
    return Y.T.copy(), res


class Hierarchy:
    """Shifted-Laplacian multigrid hierarchy (Galerkin, banded-LU coarsest)."""

    COARSE = {"lu": 0, "gmres": 1, "none": 2}

    def __init__(self, g, m, gamma, omega, beta, levels, nu_pre=None, nu_post=None, wjac=None,
                 coarse="lu", coarse_iters=20, coarse_restarts=1, cycle="V"):
        self.g = g
        self.levels = levels
        self.omega, self.beta = float(omega), float(beta)
        self._m, self._gamma = _d(m), _d(gamma)
        nu1 = np.ascontiguousarray(nu_pre if nu_pre is not None else [2] * levels, dtype=np.int32)
        nu2 = np.ascontiguousarray(nu_post if nu_post is not None else [2] * levels, dtype=np.int32)
        w = np.ascontiguousarray(wjac if wjac is not None else [0.8] * levels, dtype=np.float64)
        if np.isscalar(wjac):
            w = np.full(levels, float(wjac))
        if np.isscalar(nu_pre):
            nu1 = np.full(levels, int(nu_pre), np.int32)
        if np.isscalar(nu_post):
            nu2 = np.full(levels, int(nu_post), np.int32)
        self._keep = (nu1, nu2, w)
        self.h = lib().orc_setup(C.byref(g), _p(self._m), _p(self._gamma), omega, beta,
                                 levels, _p(nu1), _p(nu2), _p(w), self.COARSE[coarse],
                                 int(coarse_iters))
        if not self.h:
            raise RuntimeError("oracle setup failed")
        if coarse_restarts > 1:
            lib().orc_set_coarse_restarts(self.h, int(coarse_restarts))
        if cycle not in ("V", "W", "K"):
            raise ValueError("cycle must be 'V', 'W' or 'K'")
        if cycle == "W":
            lib().orc_set_cycle_w(self.h, 1)
        if cycle == "K":
            lib().orc_set_cycle_k(self.h, 1)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_free(self.h)
            self.h = None

    def level_grid(self, l):
        g = Grid()
        lib().orc_level_grid(self.h, l, C.byref(g))
        return g

    def stencil(self, l):
        g = self.level_grid(l)
        st = np.empty((npts(g), 27), np.complex128)
        lib().orc_level_stencil(self.h, l, _p(st))
        return st

    def vcycle(self, F):
        F = _c(F).reshape(-1, npts(self.g))
        U = np.empty_like(F)
        lib().orc_vcycle(self.h, F.shape[0], _p(F), _p(U))
        return U

    def coarse_solve(self, F):
        g = self.level_grid(self.levels - 1)
        F = _c(F).reshape(-1, npts(g))
        U = np.empty_like(F)
        lib().orc_coarse_solve(self.h, F.shape[0], _p(F), _p(U))
        return U

    def fgmres(self, Q, tol=1e-6, restart=5, maxit=500, prec=True, X0=None, hist=False):
        """Block FGMRES on the whole block Q [p][N]. Returns (X, iters, relres, conv[, hist])."""
        Q = _c(Q).reshape(-1, npts(self.g))
        p = Q.shape[0]
        X = np.zeros_like(Q) if X0 is None else _c(X0).reshape(Q.shape).copy()
        it = C.c_int(0)
        rr = np.empty(p)
        hh = np.zeros(maxit)
        rc = lib().orc_block_fgmres(self.h, 1 if prec else 0, p, _p(Q), _p(X),
                                    0 if X0 is None else 1, tol, restart, maxit,
                                    C.byref(it), _p(rr), _p(hh))
        out = (X, it.value, rr, rc == 0)
        if hist:
            out = out + (hh[: it.value],)
        return out


def setup_problem(prob, levels=None, **kw) -> Hierarchy:
    """Hierarchy for a ``synth.Problem``."""
    g = grid(prob.dim, prob.n, prob.h)
    L = levels or prob.levels
    return Hierarchy(g, prob.m, prob.gamma, prob.omega, prob.shift, L, **kw)


# ---------------------------------------------------------------------------
# Convolutional network of the learned coarsest-grid correction
# (channels last: [B][D][D][D][C] with x fastest; taps t = (dx+1)+3(dy+1)+9(dz+1))
# ---------------------------------------------------------------------------
def _conv_lib():
    L = lib()
    if not hasattr(L, "_conv_ready"):
        P, I, D = C.c_void_p, C.c_int, C.c_double
        L.orc_conv3d_fwd.argtypes = [I, I, I, I, P, P, P, I, P]
        L.orc_conv3d_bwd_data.argtypes = [I, I, I, I, P, P, P]
        L.orc_conv3d_bwd_weight.argtypes = [I, I, I, I, P, P, P, P]
        L.orc_avgpool2.argtypes = [I, I, I, P, P]
        L.orc_upsample2.argtypes = [I, I, I, P, P]
        L.orc_unet_nparams.restype = C.c_long
        L.orc_unet_forward.argtypes = [I, I, P, P, P]
        L.orc_unet_loss_grad.restype = D
        L.orc_unet_loss_grad.argtypes = [I, I, P, P, P, P, P]
        L._conv_ready = True
    return L


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def conv3d(x, W, b=None, relu=False):
    """x [B,D,D,D,Cin], W [27,Cin,Cout], b [Cout] -> [B,D,D,D,Cout]."""
    x, W = _f64(x), _f64(W)
    B, D, Cin, Cout = x.shape[0], x.shape[1], x.shape[4], W.shape[2]
    y = np.empty(x.shape[:4] + (Cout,))
    bb = None if b is None else _f64(b)
    _conv_lib().orc_conv3d_fwd(B, D, Cin, Cout, _p(x), _p(W), None if bb is None else _p(bb), int(relu), _p(y))
    return y


def conv3d_bwd_data(dy, W):
    dy, W = _f64(dy), _f64(W)
    B, D, Cin, Cout = dy.shape[0], dy.shape[1], W.shape[1], W.shape[2]
    dx = np.empty(dy.shape[:4] + (Cin,))
    _conv_lib().orc_conv3d_bwd_data(B, D, Cin, Cout, _p(dy), _p(W), _p(dx))
    return dx


def conv3d_bwd_weight(x, dy):
    x, dy = _f64(x), _f64(dy)
    B, D, Cin, Cout = x.shape[0], x.shape[1], x.shape[4], dy.shape[4]
    dW = np.empty((27, Cin, Cout))
    db = np.empty(Cout)
    _conv_lib().orc_conv3d_bwd_weight(B, D, Cin, Cout, _p(x), _p(dy), _p(dW), _p(db))
    return dW, db


def avgpool2(x):
    x = _f64(x)
    B, D, Cc = x.shape[0], x.shape[1], x.shape[4]
    y = np.empty((B, D // 2, D // 2, D // 2, Cc))
    _conv_lib().orc_avgpool2(B, D, Cc, _p(x), _p(y))
    return y


def upsample2(x):
    x = _f64(x)
    B, d, Cc = x.shape[0], x.shape[1], x.shape[4]
    y = np.empty((B, 2 * d, 2 * d, 2 * d, Cc))
    _conv_lib().orc_upsample2(B, d, Cc, _p(x), _p(y))
    return y


UNET_LAYERS = ((4, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (96, 32), (32, 32), (48, 16), (16, 16))


def unet_nparams():
    return int(_conv_lib().orc_unet_nparams())


def unet_forward(params, x):
    """params: packed float64 vector; x [B,D,D,D,4] -> out [B,D,D,D,2]."""
    params, x = _f64(params), _f64(x)
    B, D = x.shape[0], x.shape[1]
    out = np.empty((B, D, D, D, 2))
    _conv_lib().orc_unet_forward(B, D, _p(params), _p(x), _p(out))
    return out


def unet_loss_grad(params, x, target, mask=None):
    """Mean over samples of ||out - t||^2/||t||^2 (on mask != 0) and its gradient."""
    params, x, target = _f64(params), _f64(x), _f64(target)
    B, D = x.shape[0], x.shape[1]
    g = np.empty_like(params)
    mk = None if mask is None else _f64(mask)
    loss = _conv_lib().orc_unet_loss_grad(B, D, _p(params), _p(x), _p(target),
                                          None if mk is None else _p(mk), _p(g))
    return loss, g
