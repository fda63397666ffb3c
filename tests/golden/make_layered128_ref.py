"""Writes layered128_ref.json: sampled values of the oracle's solution of the
3D 128^3 layered workload (128^3 cells, 127^3 unknowns, 8-layer model with
a smooth perturbation, seed 2, 32 surface sources on an 8 x 4 lattice,
8 points per wavelength, 12-cell absorbing layer).

The oracle (plain FP64 C) solves two of the 32 columns with block FGMRES(5)
preconditioned by its 3-level shifted-Laplacian V-cycle with the exact
(banded LU) coarsest solve, to a relative residual of 1e-10. Stored per
column: the 2-norm of the whole solution and its values at 1024 seeded
random nodes plus the 27 nodes around the source. Only oracle/ and synth/
are called. Run from the repository root:
    python tests/golden/make_layered128_ref.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

COLUMNS = [0, 19]
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "layered128_ref.json")


def sample_nodes(p, col):
    """1024 seeded random unknowns and the 3 x 3 x 3 block around the source."""
    rng = np.random.default_rng(1000 + col)
    idx = set(int(i) for i in rng.choice(p.N, size=1024, replace=False))
    shape = tuple(c - 1 for c in p.n)[::-1]  # numpy order (z, y, x)
    z, y, x = p.src[col]
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                zz, yy, xx = z + dz, y + dy, x + dx
                if 0 <= zz < shape[0] and 0 <= yy < shape[1] and 0 <= xx < shape[2]:
                    idx.add(int(np.ravel_multi_index((zz, yy, xx), shape)))
    return sorted(idx)


def main():
    p = synth.layered_3d(n=128, seed=2, nsrc=(8, 4), levels=3)
    t0 = time.time()
    ho = oracle.setup_problem(p, levels=3)
    X, it, rr, conv = ho.fgmres(p.Q[COLUMNS], tol=1e-10, restart=5, maxit=5000)
    assert conv, rr
    cols = []
    for k, c in enumerate(COLUMNS):
        idx = sample_nodes(p, c)
        cols.append({"column": c, "norm2": float(np.linalg.norm(X[k])), "relres": float(rr[k]),
                     "nodes": idx, "re": [repr(float(v)) for v in X[k, idx].real],
                     "im": [repr(float(v)) for v in X[k, idx].imag]})
    doc = {"workload": "synth.layered_3d(n=128, seed=2, nsrc=(8, 4), levels=3)",
           "solver": "oracle block FGMRES(5), 3-level V(2,2) shifted-Laplacian (shift 0.2, Jacobi 0.8), "
                     "banded-LU coarsest, X0 = 0",
           "tol": 1e-10, "iterations": it, "threads": oracle.num_threads(),
           "seconds": round(time.time() - t0, 1), "columns": cols}
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=0)
    print("wrote", OUT, "iterations", it, "relres", rr)


if __name__ == "__main__":
    main()
