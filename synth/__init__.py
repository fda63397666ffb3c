"""Seeded synthetic inputs for the block Helmholtz solver.

This module is shared by the CPU oracle, the tests and the benchmark. It
holds no arithmetic of the solver itself: it only draws velocity models,
the absorbing-layer attenuation profile, the frequency for a points-per-
wavelength rule, and point-source right-hand sides.

Conventions (the grid of the paper's discretisation, section on the
Helmholtz forward problem): a domain of ``n`` cells per axis has nodes
0..n, of which 1..n-1 are unknowns (homogeneous Dirichlet outside).
Arrays are C-ordered with axis 0 of the *solver* fastest, i.e. numpy shape
``(nz, nx)`` in 2D and ``(nz, ny, nx)`` in 3D, z being depth. Depth index 0
of the unknowns is the first row below the free surface.

The paper's experiments use the SEG/EAGE salt model, which is not
available here; the layered models below take its velocity range
(1.5-4.5 km/s) and the points-per-wavelength rule of the multigrid
experiments instead.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem", "gradient_model_2d", "layered_model", "layer_gamma",
    "omega_for_ppw", "surface_sources", "random_rhs", "gradient_2d", "layered_3d",
    "training_model", "batch_instances", "frequency_sweep",
]


@dataclasses.dataclass
class Problem:
    """A Helmholtz instance: model, attenuation, frequency and sources."""
    dim: int
    n: tuple            # cells per axis, solver order (x, [y,] z)
    h: tuple            # spacing per axis, solver order
    m: np.ndarray       # squared slowness, float64, numpy shape (nz,[ny,]nx)
    gamma: np.ndarray   # dimensionless attenuation incl. absorbing layer
    omega: float
    Q: np.ndarray       # complex128 [nrhs][N], each RHS contiguous, x fastest
    src: list           # source node indices (numpy order tuples)
    shift: float = 0.2
    levels: int = 3
    nu_pre: int = 2
    nu_post: int = 2
    jacobi_weight: float = 0.8
    restart: int = 5
    tol: float = 1e-6
    name: str = ""

    @property
    def N(self) -> int:
        return int(np.prod([c - 1 for c in self.n]))

    @property
    def nrhs(self) -> int:
        return int(self.Q.shape[0])


def _axis_nodes(n: int) -> np.ndarray:
    """Positions (in cells) of the unknown nodes 1..n-1 along one axis."""
    return np.arange(1, n, dtype=np.float64)


def gradient_model_2d(n: int, v0: float = 1.5, v1: float = 3.0) -> np.ndarray:
    """Velocity rising linearly with depth from v0 (surface) to v1 (bottom)."""
    z = _axis_nodes(n) / n
    v = v0 + (v1 - v0) * z
    return np.repeat(v[:, None], n - 1, axis=1)


def _gaussian_smooth(a: np.ndarray, sigma: float, truncate: float = 4.0) -> np.ndarray:
    """Separable Gaussian filter with reflecting edges (scipy-free)."""
    r = int(truncate * sigma + 0.5)
    x = np.arange(-r, r + 1, dtype=np.float64)
    k = np.exp(-0.5 * (x / sigma) ** 2)
    k /= k.sum()
    out = a
    for ax in range(a.ndim):
        pad = [(0, 0)] * a.ndim
        pad[ax] = (r, r)
        p = np.pad(out, pad, mode="symmetric")
        acc = np.zeros_like(out)
        for j, w in enumerate(k):
            sl = [slice(None)] * a.ndim
            sl[ax] = slice(j, j + out.shape[ax])
            acc += w * p[tuple(sl)]
        out = acc
    return out


def layered_model(dim: int, n: int, seed: int, nlayers: int = 8,
                  vmin: float = 1.5, vmax: float = 4.5, pert: float = 0.1,
                  sigma: float = 5.0) -> np.ndarray:
    """Random layered velocity (km/s) plus a smooth random perturbation.

    ``nlayers`` layers with sorted uniform interfaces in depth and sorted
    uniform velocities in [vmin, vmax]; multiplied by (1 + p) with p a
    Gaussian-smoothed white noise rescaled to max|p| = ``pert``.
    """
    rng = np.random.default_rng(seed)
    ifc = np.sort(rng.uniform(0.0, 1.0, nlayers - 1))
    vel = np.sort(rng.uniform(vmin, vmax, nlayers))
    z = _axis_nodes(n) / n
    vz = vel[np.searchsorted(ifc, z)]
    shape = (n - 1,) * dim
    v = np.broadcast_to(vz.reshape((-1,) + (1,) * (dim - 1)), shape).copy()
    if pert > 0:
        p = _gaussian_smooth(rng.standard_normal(shape), sigma)
        p *= pert / np.abs(p).max()
        v *= 1.0 + p
    return v


def layer_gamma(dim: int, n: int, width: int, gmax: float = 0.3,
                top: bool = False, gamma0: float = 0.0) -> np.ndarray:
    """Absorbing layer: gamma = gmax * (depth into the layer / width)^2.

    The depth is measured in cells from the layer's inner edge, so it is 1
    on the (Dirichlet) boundary node itself. All faces are absorbing except
    the top (z = 0) free surface unless ``top``. ``gamma0`` is a constant
    interior attenuation added everywhere.
    """
    k = _axis_nodes(n)
    lo = np.maximum(width - k, 0.0) / width
    hi = np.maximum(k - (n - width), 0.0) / width
    both = np.maximum(lo, hi)
    zprof = both if top else hi
    if dim == 2:
        g = np.maximum(zprof[:, None], both[None, :])
    else:
        g = np.maximum(np.maximum(zprof[:, None, None], both[None, :, None]),
                       both[None, None, :])
    return gamma0 + gmax * g ** 2


def omega_for_ppw(vmin: float, ppw: float, h: float) -> float:
    """Angular frequency giving ``ppw`` grid points per shortest wavelength."""
    return 2.0 * math.pi * vmin / (ppw * h)


def _spread(count: int, n: int, width: int) -> list:
    """``count`` node indices (0-based unknowns) evenly over the non-layer span
    (over the whole axis when the layer leaves fewer than ``count`` cells)."""
    lo, hi = width, n - width
    if hi - lo < count:
        lo, hi = 0, n
    return [int(round(lo + (hi - lo) * (i + 0.5) / count)) - 1 for i in range(count)]


def surface_sources(dim: int, n: int, grid: tuple, width: int, depth: int = 0):
    """Point sources on the first unknown row below the surface.

    ``grid`` = (count along x,) in 2D or (count along x, count along y) in
    3D. Returns numpy-order index tuples.
    """
    if dim == 2:
        return [(depth, x) for x in _spread(grid[0], n, width)]
    return [(depth, y, x) for y in _spread(grid[1], n, width)
            for x in _spread(grid[0], n, width)]


def point_rhs(dim: int, n: int, h: float, src: list) -> np.ndarray:
    """Finite-volume delta: amplitude h^-dim at one node per source."""
    N = (n - 1) ** dim
    Q = np.zeros((len(src), N), dtype=np.complex128)
    shape = (n - 1,) * dim
    for s, idx in enumerate(src):
        Q[s, np.ravel_multi_index(idx, shape)] = h ** (-dim)
    return Q


def random_rhs(N: int, nrhs: int, seed: int) -> np.ndarray:
    """Dense complex Gaussian right-hand sides [nrhs][N]."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((nrhs, N)) + 1j * rng.standard_normal((nrhs, N)))


def _make(dim, n, v, width, ppw, srcgrid, name, levels, restart, top=False):
    h = 1.0 / n
    m = 1.0 / v ** 2
    gamma = layer_gamma(dim, n, width, top=top)
    omega = omega_for_ppw(float(v.min()), ppw, h)
    src = surface_sources(dim, n, srcgrid, width)
    Q = point_rhs(dim, n, h, src)
    return Problem(dim=dim, n=(n,) * dim, h=(h,) * dim, m=m, gamma=gamma,
                   omega=omega, Q=Q, src=src, levels=levels, restart=restart,
                   name=name)


def gradient_2d(n: int = 128, nsrc: tuple = (4,), levels: int = 3) -> Problem:
    """2D workload: n^2 cells (default 128^2), velocity linear in depth from
    1.5 to 3.0 km/s, 16-cell absorbing layer, 10 points per wavelength,
    sources on the first unknown row, FGMRES(10)."""
    return _make(2, n, gradient_model_2d(n), 16, 10.0, nsrc, f"gradient2d-{n}", levels, 10)


def layered_3d(n: int = 128, seed: int = 2, nsrc: tuple = (8, 4), levels: int = 4) -> Problem:
    """3D workload: n^3 cells, a seeded 8-layer velocity model (1.5-4.5 km/s)
    with a 10% smooth perturbation, 12-cell absorbing layer, 8 points per
    wavelength, an nsrc[0] x nsrc[1] lattice of surface sources, FGMRES(5).
    The 192^3 benchmark solve is layered_3d(192, seed=3, nsrc=(8, 8))."""
    return _make(3, n, layered_model(3, n, seed), 12, 8.0, nsrc, f"layered3d-{n}-s{seed}", levels, 5)


def training_model(j: int, n: int = 128, nsrc: tuple = (8, 4)) -> Problem:
    """Training model j of the learned coarsest correction: the layered 3D
    family (8 layers + 10% smooth perturbation, 12-cell layer, 8 ppw, 3
    levels) with seed 5000 + j, so that no training model is a benchmark
    model; 32 surface sources (8x4)."""
    return _make(3, n, layered_model(3, n, 5000 + j), 12, 8.0, nsrc, f"train{j}", 3, 5)


def batch_instances(count: int = 48, seed: int = 4000, sizes_2d=None, sizes_3d=None,
                    ppw: tuple = (8.0, 12.0)) -> list:
    """Independent uneven instances (the batched workload), one seed each.

    Instance k uses seed ``seed + k``. The first half are 2D with n drawn from
    64, 96, ..., 512 cells, the second half 3D with n from 64, 96, 128, 160.
    Each has 4-8 random layers (3D: plus the 10% smooth perturbation),
    ``ppw`` points per wavelength (default 8-12), a 16-cell (2D) or 12-cell
    (3D) absorbing layer and 1-32 surface sources spread along x; FGMRES(5).
    The cycle depth keeps at least 4 points per wavelength on every smoothed
    level: 3 levels from 8 points per wavelength up, 2 below.
    """
    sizes_2d = sizes_2d or list(range(64, 513, 32))
    sizes_3d = sizes_3d or [64, 96, 128, 160]
    out = []
    for k in range(count):
        rng = np.random.default_rng(seed + k)
        dim = 2 if k < count // 2 else 3
        n = int(rng.choice(sizes_2d if dim == 2 else sizes_3d))
        nl = int(rng.integers(4, 9))
        w = float(rng.uniform(*ppw))
        nsrc = int(rng.integers(1, 33))
        v = layered_model(dim, n, seed + k, nlayers=nl, pert=0.0 if dim == 2 else 0.1)
        width = 16 if dim == 2 else 12
        grid = (nsrc,) if dim == 2 else (nsrc, 1)
        out.append(_make(dim, n, v, width, w, grid, f"batch{k}", 3 if w >= 8.0 else 2, 5))
    return out



def frequency_sweep(base: Problem, freqs=(2.0, 2.5, 3.5, 4.5, 6.0)) -> list:
    """The problem at several frequencies, as frequency continuation needs:
    the same model, attenuation and sources, with omega scaled by
    freqs / max(freqs) from the base problem's omega (which thus belongs to
    the highest frequency). The default set has the ratios of the paper's
    frequency list (2.0, 2.5, 3.5, 4.5, 6.0 Hz). Instances are named by
    their ratio, lowest first."""
    fmax = max(freqs)
    out = []
    for f in sorted(freqs):
        p = dataclasses.replace(base, omega=base.omega * f / fmax, name=f"{base.name}-f{f:g}")
        out.append(p)
    return out
